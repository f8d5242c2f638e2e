// C ABI of the multiphase lattice Boltzmann library (declarations and the
// contract of every call: include/mplb.h).
//
// Device memory layout inside the caller's arena (each region 256-byte
// aligned, np = cell count rounded up to a multiple of 64):
//   F0 G0 F1 G1   populations, [Q][np] each, ping-pong pairs; Fk and Gk are
//                 adjacent so that the idle pair doubles as a staging area for
//                 host transfers
//   phi           order parameter of the current time level, [np]
//   fp, fr, gp    per-cell shift/scale of FP16-shifted sets, two of each
//   phiu          (phi u) of two steps (first-order phase-field equilibrium)
//   npart, nedge  partial sums of the next phi (lattices the summing update
//                 kernel can take; edge sized for tiles of one row)
//   partials      reduction partial sums, result
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/mplb.h"
#include "internal.h"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

#define HIPCHK(call)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(MPLB_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));     \
    } while (0)

constexpr size_t ALIGN = 256;
constexpr int RED_PARTIALS = 1024;

size_t up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// A byte range of the arena.
struct Region {
    size_t off, bytes;
};

struct Layout {
    int Q;
    long long N, np;
    size_t sF, sG, sT;
    size_t F[2], G[2], phi, ref, frest[2], grest[2], phiu[2], npart, nedge, partials, result, total;
    size_t staging_bytes;
    size_t bF, bG;  // bytes of one population set of each kind (rounded to ALIGN)
};

bool validate(const mplb_params *p, std::string &why)
{
    if (!p) return why = "params is NULL", false;
    if (p->dim != 2 && p->dim != 3) return why = "dim must be 2 or 3", false;
    for (int i = 0; i < 3; ++i)
        if (p->n[i] < 1) return why = "every lattice extent must be >= 1", false;
    if (p->dim == 2 && p->n[2] != 1) return why = "nz must be 1 in 2-D", false;
    const long long N = (long long)p->n[0] * p->n[1] * p->n[2];
    if (N > 0x7fffffffLL - 64) return why = "lattice has more than 2^31 cells", false;
    for (int i = 0; i < p->dim; ++i)
        if (p->bc[i] < MPLB_BC_PERIODIC || p->bc[i] > MPLB_BC_SYMMETRY)
            return why = "unknown boundary type", false;
    auto pos = [](double v) { return std::isfinite(v) && v > 0.0; };
    if (!pos(p->rho_heavy) || !pos(p->rho_light)) return why = "densities must be > 0", false;
    if (!pos(p->nu_heavy) || !pos(p->nu_light)) return why = "viscosities must be > 0", false;
    if (!std::isfinite(p->W) || p->W < 1.0) return why = "interface thickness W must be >= 1", false;
    if (!pos(p->mobility)) return why = "mobility must be > 0", false;
    if (!std::isfinite(p->sigma) || p->sigma < 0.0) return why = "surface tension must be >= 0", false;
    for (int i = 0; i < 3; ++i)
        if (!std::isfinite(p->gravity[i])) return why = "gravity must be finite", false;
    if (p->dim == 2 && p->gravity[2] != 0.0) return why = "gravity[2] must be 0 in 2-D", false;
    if (p->storage < MPLB_STORE_FP64 || p->storage > MPLB_STORE_FP16S_ALL)
        return why = "unknown storage format", false;
    if (p->visc_interp != 0 && p->visc_interp != 1) return why = "visc_interp must be 0 or 1", false;
    if (p->collision != MPLB_COLL_CUMULANT && p->collision != MPLB_COLL_SRT)
        return why = "unknown collision operator", false;
    if (p->cac_edf != 0 && p->cac_edf != 1) return why = "cac_edf must be 0 or 1", false;
    return true;
}

// Lattices whose update kernel can sum the next phi (see mplb::nphi_ok; the
// block shape is checked at each step).
bool nphi_geom(const mplb_params *p)
{
    auto per_or_wall = [](int b) { return b == MPLB_BC_PERIODIC || b == MPLB_BC_WALL; };
    return p->dim == 3 && p->bc[0] == MPLB_BC_PERIODIC &&
           per_or_wall(p->bc[1]) && per_or_wall(p->bc[2]) &&
           mplb::nphi_width_ok(p->n[0], p->storage);
}

Layout make_layout(const mplb_params *p)
{
    Layout L{};
    L.Q = p->dim == 2 ? 9 : 27;
    L.N = (long long)p->n[0] * p->n[1] * p->n[2];
    L.np = (L.N + 63) / 64 * 64;
    const bool f16 = p->storage == MPLB_STORE_FP16S || p->storage == MPLB_STORE_FP16S_ALL;
    L.sF = p->storage == MPLB_STORE_FP64 ? 8 : f16 ? 2 : 4;
    L.sG = p->storage == MPLB_STORE_FP64 ? 8 : p->storage == MPLB_STORE_FP16S_ALL ? 2 : 4;
    L.sT = p->storage == MPLB_STORE_FP64 ? 8 : 4;
    size_t off = 0;
    const size_t bF = up(L.Q * L.np * L.sF, ALIGN), bG = up(L.Q * L.np * L.sG, ALIGN);
    for (int k = 0; k < 2; ++k) {
        L.F[k] = off;
        off += bF;
        L.G[k] = off;
        off += bG;
    }
    L.staging_bytes = bF + bG;
    L.bF = bF;
    L.bG = bG;
    // phi of the current level; FP16 formats: 8-byte records (phi and the
    // cell's packed references), the reference array the update writes, and
    // the rest-direction values of each FP16 set in FP32, two levels
    L.phi = off;
    off += up(L.np * (f16 ? 8 : L.sT), ALIGN);
    const size_t b4 = up(L.np * 4, ALIGN);
    L.ref = 0;
    if (f16) {
        L.ref = off;
        off += b4;
    }
    for (int k = 0; k < 2; ++k) {
        L.frest[k] = L.grest[k] = 0;
        if (f16) {
            L.frest[k] = off;
            off += b4;
        }
        if (p->storage == MPLB_STORE_FP16S_ALL) {
            L.grest[k] = off;
            off += b4;
        }
    }
    // (phi u) of the current and previous step, [3][np] in the arithmetic
    // type, for the first-order phase-field equilibrium only
    for (int k = 0; k < 2; ++k) {
        L.phiu[k] = 0;
        if (p->cac_edf) {
            L.phiu[k] = off;
            off += up(3 * L.np * L.sT, ALIGN);
        }
    }
    L.npart = L.nedge = 0;
    if (nphi_geom(p)) {
        L.npart = off;
        off += up(3 * L.np * L.sT, ALIGN);
        L.nedge = off;
        off += up(6 * L.N * L.sT, ALIGN);  // enough for tiles of one row
    }
    L.partials = off;
    off += up(RED_PARTIALS * 8 * sizeof(double), ALIGN);
    L.result = off;
    off += up(8 * sizeof(double), ALIGN);
    L.total = off;
    return L;
}

// Default block: as wide in x as the lattice (up to 256 cells) so that the
// cache lines split by the x-shifted pulls stay inside one workgroup, then
// filled along y and z to 256 threads.
dim3 default_block(const mplb_params *p)
{
    auto pow2 = [](int v, int cap) {
        int b = 1;
        while (b < v && b < cap) b <<= 1;
        return b;
    };
    const int bx = pow2(p->n[0], 256);
    const int by = pow2(p->n[1], 256 / bx);
    const int bz = pow2(p->n[2], 256 / (bx * by));
    return dim3(bx, by, bz);
}

mplb::PhysD make_phys(const mplb_params *p)
{
    mplb::PhysD d{};
    d.rho_l = p->rho_light;
    d.drho = p->rho_heavy - p->rho_light;
    d.nu_l = p->nu_light;
    d.dnu = p->nu_heavy - p->nu_light;
    d.rnu_l = p->rho_light * p->nu_light;
    d.drnu = p->rho_heavy * p->nu_heavy - p->rho_light * p->nu_light;
    d.beta = 12.0 * p->sigma / p->W;
    d.kappa = 1.5 * p->sigma * p->W;
    d.gx = p->gravity[0];
    d.gy = p->gravity[1];
    d.gz = p->dim == 3 ? p->gravity[2] : 0.0;
    const double tpb = p->mobility * 3.0 + 0.5;
    d.inv_tpb = 1.0 / tpb;
    d.src_pre = 1.0 - 0.5 / tpb;
    d.four_W = 4.0 / p->W;
    d.scl_l = p->rho_light / 3.0;
    d.dscl = (p->rho_heavy - p->rho_light) / 3.0;
    d.visc_interp = p->visc_interp;
    d.collision = p->collision;
    d.cac_edf = p->cac_edf;
    return d;
}

}  // namespace

struct mplb_solver {
    mplb_params prm;
    Layout L;
    char *base;
    hipStream_t stream;
    int cur;
    int64_t steps;
    bool ready;
    bool attached;
    bool hist;  // (phi u) of the previous step is stored (first-order phase-field equilibrium)
    int nphi;  // update kernel that sums the next phi: 0 never, 1 where it applies
    bool nphi_valid;  // the last update wrote partial sums of the current phi
    dim3 block;
    mplb::PhysD ph;
    // Steps replayed as a captured graph (mplb_step): GRAPH_STEPS steps from
    // level g_cur with block g_block and the phi-summing update on or off
    // (g_nphi), captured on a private stream at the default priority.
    hipStream_t cap;
    hipGraphExec_t gexec;
    bool have_g;
    int g_cur;
    dim3 g_block;
    bool g_nphi;

    mplb_solver() = default;
    mplb_solver(const mplb_solver &) = delete;
    mplb_solver &operator=(const mplb_solver &) = delete;
    ~mplb_solver()
    {
        // replays still in flight finish before their graph goes
        if (have_g) (void)hipStreamSynchronize(stream);
        drop_graph();
        if (cap) (void)hipStreamDestroy(cap);
    }
    void drop_graph()
    {
        if (have_g) (void)hipGraphExecDestroy(gexec);
        have_g = false;
    }

    void *at(size_t off) const { return off ? base + off : nullptr; }
    bool use_nphi(const mplb::Ctx &c) const
    {
        return nphi != 0 && L.npart != 0 && mplb::nphi_ok(c);
    }
    mplb::NextPhi next_phi() const
    {
        return mplb::NextPhi{at(L.npart), at(L.nedge),
                             mplb::nphi_rows(prm.n[0], prm.n[1], prm.storage)};
    }
    // The phi stage of a step: merge the partial sums the previous update
    // wrote, or sum the pulled populations.
    hipError_t launch_phi_stage(const mplb::Ctx &c) const
    {
        if (use_nphi(c) && nphi_valid) return mplb::launch_phi_merge(c, next_phi());
        return mplb::launch_phi(c);
    }
    // The update stage; records whether it left partial sums for the next step.
    hipError_t launch_update_stage(const mplb::Ctx &c)
    {
        nphi_valid = use_nphi(c);
        return nphi_valid ? mplb::launch_collide_nphi(c, next_phi()) : mplb::launch_collide(c);
    }
    void *F(int k) const { return base + L.F[k]; }
    void *G(int k) const { return base + L.G[k]; }
    double *staging(int k) const { return reinterpret_cast<double *>(base + L.F[k]); }

    // Context for work that reads buffer `in` and writes buffer 1 - in.
    mplb::Ctx ctx(int in) const
    {
        mplb::Ctx c{};
        c.dim = prm.dim;
        c.storage = prm.storage;
        c.g.nx = prm.n[0];
        c.g.ny = prm.n[1];
        c.g.nz = prm.n[2];
        c.g.bcx = prm.bc[0];
        c.g.bcy = prm.bc[1];
        c.g.bcz = prm.dim == 3 ? prm.bc[2] : mplb::BC_PER;
        c.g.np = L.np;
        c.ph = ph;
        c.block = block;
        c.stream = stream;
        c.p.Fin = F(in);
        c.p.Gin = G(in);
        c.p.Fout = F(1 - in);
        c.p.Gout = G(1 - in);
        c.p.phi = base + L.phi;
        c.p.ref = static_cast<unsigned *>(at(L.ref));
        c.p.frest_in = static_cast<const float *>(at(L.frest[in]));
        c.p.grest_in = static_cast<const float *>(at(L.grest[in]));
        c.p.frest_out = static_cast<float *>(at(L.frest[1 - in]));
        c.p.grest_out = static_cast<float *>(at(L.grest[1 - in]));
        c.p.phiu_in = at(L.phiu[in]);
        c.p.phiu_out = at(L.phiu[1 - in]);
        c.p.have_prev = hist ? 1 : 0;
        return c;
    }

    // Device regions a step from the current state reads (see save / load).
    std::vector<Region> state_regions() const { return state_regions(cur, nphi_valid); }
    // The same for a state at level k whose partial sums are valid or not.
    std::vector<Region> state_regions(int k, bool with_partials) const
    {
        std::vector<Region> r;
        r.push_back({L.F[k], L.bF});
        r.push_back({L.G[k], L.bG});
        const size_t b4 = up(L.np * 4, ALIGN);
        if (L.ref) r.push_back({L.ref, b4});
        if (L.frest[k]) r.push_back({L.frest[k], b4});
        if (L.grest[k]) r.push_back({L.grest[k], b4});
        if (L.phiu[k]) r.push_back({L.phiu[k], size_t(3) * L.np * L.sT});
        if (with_partials) {
            r.push_back({L.npart, size_t(3) * L.np * L.sT});
            const mplb::NextPhi q = next_phi();
            r.push_back({L.nedge, size_t(6) * (prm.n[1] / q.by) * prm.n[2] * prm.n[0] * L.sT});
        }
        return r;
    }

    // Context that writes (in place) into buffer k.
    mplb::Ctx ctx_write(int k) const
    {
        mplb::Ctx c = ctx(1 - k);
        return c;
    }
};

namespace {

// ------------------------------------------------------------ save / load
// A saved state is a host blob: a header (format, parameters, the handle's
// step bookkeeping and launch settings), a table of region sizes, then the
// raw device bytes of every region a following step reads: the population
// buffers of the current level (as stored, FP16 codes included), the
// per-cell references of the shifted formats, the (phi u) history of the
// first-order phase-field equilibrium, and the partial sums of phi when the
// last update wrote them.  Loading them back into a solver with equal
// parameters reproduces the saved solver's later steps bit for bit.
constexpr char SAVE_MAGIC[8] = {'M', 'P', 'L', 'B', 'S', 'A', 'V', 'E'};
constexpr uint32_t SAVE_FORMAT = 1;
constexpr int SAVE_MAX_REGIONS = 16;

struct SaveHeader {
    char magic[8];
    uint32_t format, nregions;
    uint64_t param_hash;
    int64_t steps;
    int32_t cur, hist, nphi, nphi_valid, ready;
    int32_t block[3];
};

// FNV-1a over the parameter values (not the struct's padding bytes).
uint64_t param_hash(const mplb_params &p)
{
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](const void *v, size_t n) {
        const unsigned char *c = static_cast<const unsigned char *>(v);
        for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
    };
    mix(&p.dim, 4);
    mix(p.n, 12);
    mix(p.bc, 12);
    const double d[] = {p.rho_heavy, p.rho_light, p.nu_heavy, p.nu_light, p.W, p.mobility,
                        p.sigma, p.gravity[0], p.gravity[1], p.gravity[2]};
    mix(d, sizeof(d));
    const int32_t k[] = {p.storage, p.visc_interp, p.collision, p.cac_edf};
    mix(k, sizeof(k));
    return h;
}

}  // namespace

extern "C" {

int32_t mplb_version(void) { return MPLB_VERSION; }

const char *mplb_arch(void) { return "gfx950"; }

const char *mplb_last_error(void) { return g_err.c_str(); }

size_t mplb_state_bytes(const mplb_params *p)
{
    std::string why;
    if (!validate(p, why)) {
        g_err = why;
        return 0;
    }
    return make_layout(p).total;
}

int mplb_create(const mplb_params *p, void *dev_arena, size_t arena_bytes, void *hip_stream,
                mplb_solver **out)
{
    std::string why;
    if (!out) return fail(MPLB_EINVAL, "out is NULL");
    *out = nullptr;
    if (!validate(p, why)) return fail(MPLB_EINVAL, why);
    if (!dev_arena) return fail(MPLB_EINVAL, "arena is NULL");
    if (reinterpret_cast<uintptr_t>(dev_arena) % ALIGN)
        return fail(MPLB_EINVAL, "arena must be 256-byte aligned");
    const Layout L = make_layout(p);
    if (arena_bytes < L.total)
        return fail(MPLB_ENOMEM, "arena holds " + std::to_string(arena_bytes) + " bytes, " +
                                     std::to_string(L.total) + " needed");
    mplb_solver *s = new (std::nothrow) mplb_solver();
    if (!s) return fail(MPLB_ENOMEM, "host allocation failed");
    s->prm = *p;
    s->L = L;
    s->base = static_cast<char *>(dev_arena);
    s->stream = static_cast<hipStream_t>(hip_stream);
    s->cur = 0;
    s->steps = 0;
    s->ready = false;
    s->attached = false;
    s->block = default_block(p);
    s->nphi = 1;
    s->nphi_valid = false;
    s->ph = make_phys(p);
    *out = s;
    return MPLB_OK;
}

void mplb_destroy(mplb_solver *s) { delete s; }

int mplb_tune_block(mplb_solver *s, int32_t steps, const int32_t *candidates, int32_t ncand,
                    int32_t best[3], double *best_ms_per_step)
{
    static const int32_t builtin3[] = {64, 4, 1, 64, 2, 2, 64, 1, 4, 32, 8, 1, 32, 4, 2,
                                       128, 2, 1, 128, 1, 2, 256, 1, 1, 64, 2, 1, 32, 2, 2};
    static const int32_t builtin2[] = {64, 4, 1, 32, 8, 1, 128, 2, 1, 256, 1, 1, 64, 2, 1,
                                       16, 16, 1, 128, 1, 1};
    if (!s || !best || !best_ms_per_step) return fail(MPLB_EINVAL, "solver and outputs are required");
    if (steps < 1) return fail(MPLB_EINVAL, "steps must be >= 1");
    if (s->attached) return fail(MPLB_ESTATE, "solver is attached to a batch");
    if (!candidates) {
        candidates = s->prm.dim == 3 ? builtin3 : builtin2;
        ncand = s->prm.dim == 3 ? int32_t(sizeof(builtin3) / 12) : int32_t(sizeof(builtin2) / 12);
    }
    const dim3 keep = s->block;
    double best_ms = 1e300;
    for (int i = 0; i < ncand; ++i) {
        const int32_t *c = candidates + 3 * i;
        if (s->prm.dim == 2 && c[2] != 1) continue;
        if (mplb_set_block(s, c[0], c[1], c[2]) != MPLB_OK) continue;
        double a = 0, b = 0;
        int rc = mplb_step_timed(s, 2, &a, &b);
        if (rc == MPLB_OK) rc = mplb_step_timed(s, steps, &a, &b);
        if (rc != MPLB_OK) {
            s->block = keep;
            return rc;
        }
        const double ms = (a + b) / steps;
        if (ms < best_ms) {
            best_ms = ms;
            best[0] = c[0];
            best[1] = c[1];
            best[2] = c[2];
        }
    }
    if (best_ms == 1e300) {
        s->block = keep;
        return fail(MPLB_EINVAL, "no valid candidate block shape");
    }
    s->block = dim3(best[0], best[1], best[2]);
    *best_ms_per_step = best_ms;
    return MPLB_OK;
}

int mplb_set_phi_partials(mplb_solver *s, int32_t mode)
{
    if (!s) return fail(MPLB_EINVAL, "solver is NULL");
    if (s->attached) return fail(MPLB_ESTATE, "solver is attached to a batch");
    if (mode != 0 && mode != 1) return fail(MPLB_EINVAL, "mode must be 0 or 1");
    s->nphi = mode;
    return MPLB_OK;
}

int mplb_uses_phi_partials(const mplb_solver *s)
{
    if (!s) return fail(MPLB_EINVAL, "solver is NULL");
    return s->use_nphi(s->ctx(s->cur)) ? s->next_phi().by : 0;
}

int mplb_set_block(mplb_solver *s, int32_t bx, int32_t by, int32_t bz)
{
    if (!s) return fail(MPLB_EINVAL, "solver is NULL");
    if (bx == 0 && by == 0 && bz == 0) {
        s->block = default_block(&s->prm);
        return MPLB_OK;
    }
    if (bx < 1 || by < 1 || bz < 1 || (long long)bx * by * bz > 256)
        return fail(MPLB_EINVAL, "block must have between 1 and 256 threads");
    if (s->prm.dim == 2 && bz != 1) return fail(MPLB_EINVAL, "bz must be 1 in 2-D");
    s->block = dim3(bx, by, bz);
    return MPLB_OK;
}

int mplb_init(mplb_solver *s, const double *phi, const double *u, const double *p)
{
    if (!s || !phi || !u) return fail(MPLB_EINVAL, "solver, phi and u are required");
    if (s->attached) return fail(MPLB_ESTATE, "solver is attached to a batch");
    const long long N = s->L.N;
    const size_t nb = N * sizeof(double);
    // inputs staged as FP64 in buffer 1: phi, u (dim components), p
    double *st = s->staging(1);
    double *dphi = st, *du = st + N, *dp = st + (1 + s->prm.dim) * N;
    HIPCHK(hipMemcpyAsync(dphi, phi, nb, hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipMemcpyAsync(du, u, nb * s->prm.dim, hipMemcpyHostToDevice, s->stream));
    if (p)
        HIPCHK(hipMemcpyAsync(dp, p, nb, hipMemcpyHostToDevice, s->stream));
    else
        HIPCHK(hipMemsetAsync(dp, 0, nb, s->stream));
    const mplb::Ctx c = s->ctx_write(0);
    if (c.p.ref) HIPCHK(mplb::launch_set_refs(c, dphi, dp));
    HIPCHK(mplb::launch_init(c, dphi, du, dp));
    HIPCHK(hipStreamSynchronize(s->stream));
    s->cur = 0;
    s->steps = 0;
    s->ready = true;
    s->hist = false;
    s->nphi_valid = false;
    return MPLB_OK;
}

namespace {

// Steps per captured graph of mplb_step: even, so that the level parity the
// graph's arguments were taken at returns after each replay.
constexpr int GRAPH_STEPS = 16;

// GRAPH_STEPS steps of the steady state (the (phi u) history present; the phi
// stage takes the same form every step) as one graph launch on the solver's
// stream.  The graph is captured once per (level parity, block, step form) on
// the solver's private stream; its kernels are those of a direct step with
// the same arguments, so the results are the same bits.
int replay_steps(mplb_solver *s)
{
    const bool nphi_now = s->use_nphi(s->ctx(s->cur));
    if (s->have_g && (s->g_cur != s->cur || s->g_block.x != s->block.x || s->g_block.y != s->block.y ||
                      s->g_block.z != s->block.z || s->g_nphi != nphi_now))
        s->drop_graph();
    if (!s->have_g) {
        if (!s->cap) HIPCHK(hipStreamCreate(&s->cap));
        HIPCHK(hipStreamBeginCapture(s->cap, hipStreamCaptureModeThreadLocal));
        hipError_t e = hipSuccess;
        int cur = s->cur;
        for (int k = 0; k < GRAPH_STEPS && e == hipSuccess; ++k) {
            mplb::Ctx c = s->ctx(cur);
            c.stream = s->cap;
            e = s->launch_phi_stage(c);
            if (e == hipSuccess) e = s->launch_update_stage(c);
            cur ^= 1;
        }
        hipGraph_t graph = nullptr;
        // always end the capture, so that a failure leaves the stream usable
        const hipError_t e2 = hipStreamEndCapture(s->cap, &graph);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return fail(MPLB_EDEVICE, std::string("step graph capture: ") +
                                          hipGetErrorString(e != hipSuccess ? e : e2));
        }
        e = hipGraphInstantiate(&s->gexec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess)
            return fail(MPLB_EDEVICE, std::string("step graph instantiate: ") + hipGetErrorString(e));
        s->have_g = true;
        s->g_cur = s->cur;
        s->g_block = s->block;
        s->g_nphi = nphi_now;
    }
    HIPCHK(hipGraphLaunch(s->gexec, s->stream));
    return MPLB_OK;
}

}  // namespace

int mplb_step(mplb_solver *s, int64_t nsteps)
{
    if (!s) return fail(MPLB_EINVAL, "solver is NULL");
    if (nsteps < 0) return fail(MPLB_EINVAL, "nsteps must be >= 0");
    if (!s->ready) return fail(MPLB_ESTATE, "mplb_init has not been called");
    if (s->attached) return fail(MPLB_ESTATE, "solver is attached to a batch");
    for (int64_t i = 0; i < nsteps;) {
        const mplb::Ctx c = s->ctx(s->cur);
        const bool steady = s->hist && (!s->use_nphi(c) || s->nphi_valid);
        if (steady && nsteps - i >= GRAPH_STEPS) {
            const int rc = replay_steps(s);
            if (rc != MPLB_OK) return rc;
            s->steps += GRAPH_STEPS;
            i += GRAPH_STEPS;
            continue;
        }
        HIPCHK(s->launch_phi_stage(c));
        HIPCHK(s->launch_update_stage(c));
        s->cur ^= 1;
        s->steps++;
        s->hist = true;
        ++i;
    }
    return MPLB_OK;
}

int mplb_step_timed(mplb_solver *s, int64_t nsteps, double *ms_phi, double *ms_collide)
{
    if (!s || !ms_phi || !ms_collide) return fail(MPLB_EINVAL, "solver and outputs are required");
    if (nsteps < 0) return fail(MPLB_EINVAL, "nsteps must be >= 0");
    if (!s->ready) return fail(MPLB_ESTATE, "mplb_init has not been called");
    if (s->attached) return fail(MPLB_ESTATE, "solver is attached to a batch");
    constexpr int BATCH = 64;
    hipEvent_t ev[2 * BATCH + 1];
    for (auto &e : ev) HIPCHK(hipEventCreate(&e));
    double tphi = 0.0, tcol = 0.0;
    int rc = MPLB_OK;
    for (int64_t done = 0; done < nsteps && rc == MPLB_OK;) {
        const int k = int(nsteps - done < BATCH ? nsteps - done : BATCH);
        hipError_t e = hipEventRecord(ev[0], s->stream);
        for (int i = 0; i < k && e == hipSuccess; ++i) {
            const mplb::Ctx c = s->ctx(s->cur);
            e = s->launch_phi_stage(c);
            if (e == hipSuccess) e = hipEventRecord(ev[2 * i + 1], s->stream);
            if (e == hipSuccess) e = s->launch_update_stage(c);
            if (e == hipSuccess) e = hipEventRecord(ev[2 * i + 2], s->stream);
            s->cur ^= 1;
            s->steps++;
            s->hist = true;
        }
        if (e == hipSuccess) e = hipEventSynchronize(ev[2 * k]);
        for (int i = 0; i < k && e == hipSuccess; ++i) {
            float a = 0.f, b = 0.f;
            e = hipEventElapsedTime(&a, ev[2 * i], ev[2 * i + 1]);
            if (e == hipSuccess) e = hipEventElapsedTime(&b, ev[2 * i + 1], ev[2 * i + 2]);
            tphi += a;
            tcol += b;
        }
        if (e != hipSuccess) rc = fail(MPLB_EDEVICE, std::string("timed step: ") + hipGetErrorString(e));
        done += k;
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    *ms_phi = tphi;
    *ms_collide = tcol;
    return rc;
}

int mplb_sync(mplb_solver *s)
{
    if (!s) return fail(MPLB_EINVAL, "solver is NULL");
    HIPCHK(hipStreamSynchronize(s->stream));
    return MPLB_OK;
}

int64_t mplb_steps_done(const mplb_solver *s) { return s ? s->steps : -1; }

int mplb_read(mplb_solver *s, int32_t field, double *host_out)
{
    if (!s || !host_out) return fail(MPLB_EINVAL, "solver and host_out are required");
    if (field < MPLB_FIELD_PHI || field > MPLB_FIELD_P) return fail(MPLB_EINVAL, "unknown field");
    if (!s->ready) return fail(MPLB_ESTATE, "mplb_init has not been called");
    if (s->prm.dim == 2 && field == MPLB_FIELD_UZ) {
        std::memset(host_out, 0, s->L.N * sizeof(double));
        return MPLB_OK;
    }
    const mplb::Ctx c = s->ctx(s->cur);
    double *st = s->staging(1 - s->cur);
    HIPCHK(mplb::launch_phi(c));
    HIPCHK(mplb::launch_field(c, field, st));
    HIPCHK(hipMemcpyAsync(host_out, st, s->L.N * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return MPLB_OK;
}

int mplb_reduce(mplb_solver *s, double out[5])
{
    if (!s || !out) return fail(MPLB_EINVAL, "solver and out are required");
    if (!s->ready) return fail(MPLB_ESTATE, "mplb_init has not been called");
    const mplb::Ctx c = s->ctx(s->cur);
    double *partials = reinterpret_cast<double *>(s->base + s->L.partials);
    double *res = reinterpret_cast<double *>(s->base + s->L.result);
    double host[8];
    HIPCHK(mplb::launch_phi(c));
    HIPCHK(mplb::launch_reduce(c, partials, res));
    HIPCHK(hipMemcpyAsync(host, res, 6 * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    for (int k = 0; k < 5; ++k) out[k] = host[k];
    if (host[5] != 0.0) return fail(MPLB_EUNSTABLE, "non-finite values in the state");
    return MPLB_OK;
}

int mplb_reduce_noalloc(mplb_solver *s, double out[5])
{
    if (!s || !out) return fail(MPLB_EINVAL, "solver and out are required");
    if (!s->ready) return fail(MPLB_ESTATE, "mplb_init has not been called");
    const mplb::Ctx c = s->ctx(s->cur);
    if (mplb::reduce_blocks(c) > mplb::reduce_scratch_max_blocks())
        return fail(MPLB_EINVAL, "the reduction needs " + std::to_string(mplb::reduce_blocks(c)) +
                                     " partial blocks, the static scratch holds " +
                                     std::to_string(mplb::reduce_scratch_max_blocks()));
    double *res = nullptr;
    double host[8];
    HIPCHK(mplb::launch_phi(c));
    HIPCHK(mplb::launch_reduce_static(c, &res));
    HIPCHK(hipMemcpyAsync(host, res, 6 * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    for (int k = 0; k < 5; ++k) out[k] = host[k];
    if (host[5] != 0.0) return fail(MPLB_EUNSTABLE, "non-finite values in the state");
    return MPLB_OK;
}

int mplb_get_populations(mplb_solver *s, int32_t which, double *host_out)
{
    if (!s || !host_out) return fail(MPLB_EINVAL, "solver and host_out are required");
    if (which != 0 && which != 1) return fail(MPLB_EINVAL, "which must be 0 (f') or 1 (g)");
    if (!s->ready) return fail(MPLB_ESTATE, "mplb_init has not been called");
    const long long N = s->L.N;
    const int chunk = int(s->L.staging_bytes / (N * sizeof(double)));
    const mplb::Ctx c = s->ctx(s->cur);
    double *st = s->staging(1 - s->cur);
    for (int a0 = 0; a0 < s->L.Q; a0 += chunk) {
        const int a1 = a0 + chunk < s->L.Q ? a0 + chunk : s->L.Q;
        HIPCHK(mplb::launch_get_pop(c, which, a0, a1, st));
        HIPCHK(hipMemcpyAsync(host_out + (long long)a0 * N, st, (a1 - a0) * N * sizeof(double),
                              hipMemcpyDeviceToHost, s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
    }
    return MPLB_OK;
}

int mplb_set_populations(mplb_solver *s, int32_t which, const double *host_in)
{
    if (!s || !host_in) return fail(MPLB_EINVAL, "solver and host_in are required");
    if (which != 0 && which != 1) return fail(MPLB_EINVAL, "which must be 0 (f') or 1 (g)");
    if (s->attached) return fail(MPLB_ESTATE, "solver is attached to a batch");
    const bool shifted = which == 0 ? s->L.sF == 2 : s->L.sG == 2;
    if (shifted && !s->ready)
        return fail(MPLB_ESTATE, "FP16-shifted sets keep the shift/scale of the current state: "
                                 "call mplb_init first");
    const long long N = s->L.N;
    const int chunk = int(s->L.staging_bytes / (N * sizeof(double)));
    // write in place into the current buffer; stage through the idle one
    const mplb::Ctx c = s->ctx_write(s->cur);
    double *st = s->staging(1 - s->cur);
    for (int a0 = 0; a0 < s->L.Q; a0 += chunk) {
        const int a1 = a0 + chunk < s->L.Q ? a0 + chunk : s->L.Q;
        HIPCHK(hipMemcpyAsync(st, host_in + (long long)a0 * N, (a1 - a0) * N * sizeof(double),
                              hipMemcpyHostToDevice, s->stream));
        HIPCHK(mplb::launch_set_pop(c, which, a0, a1, st));
        HIPCHK(hipStreamSynchronize(s->stream));
    }
    s->ready = true;
    s->steps = 0;
    s->hist = false;
    s->nphi_valid = false;
    return MPLB_OK;
}

size_t mplb_save_bytes(const mplb_solver *s)
{
    if (!s) return 0;
    size_t n = sizeof(SaveHeader) + sizeof(mplb_params) + SAVE_MAX_REGIONS * sizeof(uint64_t);
    for (const Region &r : s->state_regions()) n += r.bytes;
    return n;
}

int mplb_save(mplb_solver *s, void *host_blob, size_t bytes)
{
    if (!s || !host_blob) return fail(MPLB_EINVAL, "solver and blob are required");
    if (!s->ready) return fail(MPLB_ESTATE, "mplb_init has not been called");
    const size_t need = mplb_save_bytes(s);
    if (bytes < need)
        return fail(MPLB_EINVAL, "blob holds " + std::to_string(bytes) + " bytes, " +
                                     std::to_string(need) + " needed");
    const std::vector<Region> reg = s->state_regions();
    char *out = static_cast<char *>(host_blob);
    SaveHeader h{};
    std::memcpy(h.magic, SAVE_MAGIC, 8);
    h.format = SAVE_FORMAT;
    h.nregions = uint32_t(reg.size());
    h.param_hash = param_hash(s->prm);
    h.steps = s->steps;
    h.cur = s->cur;
    h.hist = s->hist;
    h.nphi = s->nphi;
    h.nphi_valid = s->nphi_valid;
    h.ready = s->ready;
    h.block[0] = int32_t(s->block.x);
    h.block[1] = int32_t(s->block.y);
    h.block[2] = int32_t(s->block.z);
    std::memcpy(out, &h, sizeof(h));
    std::memcpy(out + sizeof(h), &s->prm, sizeof(mplb_params));
    uint64_t sizes[SAVE_MAX_REGIONS] = {};
    for (size_t i = 0; i < reg.size(); ++i) sizes[i] = reg[i].bytes;
    std::memcpy(out + sizeof(h) + sizeof(mplb_params), sizes, sizeof(sizes));
    char *pos = out + sizeof(h) + sizeof(mplb_params) + sizeof(sizes);
    for (const Region &r : reg) {
        HIPCHK(hipMemcpyAsync(pos, s->base + r.off, r.bytes, hipMemcpyDeviceToHost, s->stream));
        pos += r.bytes;
    }
    HIPCHK(hipStreamSynchronize(s->stream));
    return MPLB_OK;
}

int mplb_load(mplb_solver *s, const void *host_blob, size_t bytes)
{
    if (!s || !host_blob) return fail(MPLB_EINVAL, "solver and blob are required");
    if (s->attached) return fail(MPLB_ESTATE, "solver is attached to a batch");
    const char *in = static_cast<const char *>(host_blob);
    constexpr size_t head = sizeof(SaveHeader) + sizeof(mplb_params) + SAVE_MAX_REGIONS * sizeof(uint64_t);
    if (bytes < head) return fail(MPLB_EINVAL, "blob is shorter than its header");
    SaveHeader h;
    std::memcpy(&h, in, sizeof(h));
    if (std::memcmp(h.magic, SAVE_MAGIC, 8) != 0 || h.format != SAVE_FORMAT)
        return fail(MPLB_EINVAL, "not a saved state of this library version");
    if (h.param_hash != param_hash(s->prm))
        return fail(MPLB_EINVAL, "saved state belongs to other parameters");
    if (h.nregions > SAVE_MAX_REGIONS || (h.cur != 0 && h.cur != 1) || h.steps < 0 ||
        (h.nphi != 0 && h.nphi != 1) || h.block[0] < 1 || h.block[1] < 1 || h.block[2] < 1 ||
        (long long)h.block[0] * h.block[1] * h.block[2] > 256)
        return fail(MPLB_EINVAL, "corrupt saved state header");
    uint64_t sizes[SAVE_MAX_REGIONS];
    std::memcpy(sizes, in + sizeof(h) + sizeof(mplb_params), sizeof(sizes));
    // the regions the saved bookkeeping implies, on this solver's layout
    const std::vector<Region> reg = s->state_regions(h.cur, h.nphi_valid != 0);
    size_t total = head;
    if (reg.size() != h.nregions) return fail(MPLB_EINVAL, "saved state does not match the layout");
    for (size_t i = 0; i < reg.size(); ++i) {
        if (sizes[i] != reg[i].bytes) return fail(MPLB_EINVAL, "saved state does not match the layout");
        total += reg[i].bytes;
    }
    if (bytes < total) return fail(MPLB_EINVAL, "blob is truncated");
    const char *pos = in + head;
    for (const Region &r : reg) {
        HIPCHK(hipMemcpyAsync(s->base + r.off, pos, r.bytes, hipMemcpyHostToDevice, s->stream));
        pos += r.bytes;
    }
    HIPCHK(hipStreamSynchronize(s->stream));
    s->cur = h.cur;
    s->steps = h.steps;
    s->hist = h.hist != 0;
    s->nphi = h.nphi;
    s->nphi_valid = h.nphi_valid != 0;
    s->ready = h.ready != 0;
    s->block = dim3(h.block[0], h.block[1], h.block[2]);
    return MPLB_OK;
}


}  // extern "C"

/* ------------------------------------------------------------------ batches */

struct mplb_batch {
    int dim, storage, collision, capacity;
    long long max_tiles;
    hipStream_t stream;
    mplb::BatchDom *d_doms;
    mplb::BatchTile *d_tiles;
    int *d_ntiles;
    long long *d_tbase;
    int *d_status;  // per slot: non-zero once the phi stage met a non-finite value
    std::vector<mplb_solver *> slot;
    std::vector<mplb::BatchDom> doms;
    std::vector<mplb::BatchTile> tiles;
    // tile list: [0, ntiles_host) block tiles of the domains updated by the
    // block kernels (phi stage and update); [ntiles_host, ntiles_phi_host)
    // block tiles of the phi-summing domains (phi stage only); then
    // ntiles_nphi_host tiles of the phi-summing update
    int ntiles_host, ntiles_phi_host, ntiles_nphi_host;
    int counts[2 + 2 * mplb::NPHI_GROUPS];  // the device tile counters (see launch_batch_step)
    int grid[2 + mplb::NPHI_GROUPS];  // blocks of the phi, update and phi-summing update
                                      // launches: tile counts rounded up to buckets of 4096
                                      // (0 for an empty group)
    dim3 block;
    int chunk;
    bool row;     // row-form kernels (see row_form_ok)
    long long t;  // batch steps taken
    hipGraphExec_t exec;
    bool have_graph;
    // Domains of at least solo_min cells fill the GPU on their own: they
    // step with their solver's own kernels (kernel arguments, no table
    // reads) on the solvers' stream, while the others share the batched
    // launches on `side`, so that the two overlap.  The streams meet at the
    // start and the end of every mplb_batch_step.
    long long solo_min;
    std::vector<char> solo;         // per slot
    std::vector<long long> start;   // per slot: the batch step it was attached at
    int nshared;                    // attached slots in the batched launches
    hipStream_t side;
    hipEvent_t ev_main, ev_side;
};

namespace {

size_t table_layout(int32_t capacity, int64_t max_tiles, size_t *o_doms, size_t *o_tiles,
                    size_t *o_nt, size_t *o_tb, size_t *o_st)
{
    size_t off = 0;
    *o_doms = off;
    off += up(sizeof(mplb::BatchDom) * capacity, ALIGN);
    *o_tiles = off;
    off += up(sizeof(mplb::BatchTile) * max_tiles, ALIGN);
    *o_nt = off;
    off += ALIGN;
    *o_tb = off;
    off += ALIGN;
    *o_st = off;
    off += up(sizeof(int) * capacity, ALIGN);
    return off;
}

void drop_graph(mplb_batch *b)
{
    if (b->have_graph) (void)hipGraphExecDestroy(b->exec);
    b->have_graph = false;
}

// Rebuild the tile list from the attached solvers and upload it with the
// domain table; synchronises the stream so the host copies can be reused.
int upload_tables(mplb_batch *b)
{
    b->tiles.clear();
    // domains whose update sums the next phi, as their solver's own step
    // would
    b->nshared = 0;
    for (int i = 0; i < b->capacity; ++i) {
        mplb_solver *s = b->slot[i];
        if (!s || b->solo[i]) continue;
        ++b->nshared;
        mplb::BatchDom &d = b->doms[i];
        const mplb::Ctx c = s->ctx(s->cur);
        const int by = (b->dim == 3 && s->use_nphi(c)) ? s->next_phi().by : 0;
        if (by != d.nphi_by) {
            d.nphi_by = by;
            d.nphi_from = b->t + 1;  // no partial sums of the current phi yet
        }
        d.npart = by ? s->at(s->L.npart) : nullptr;
        d.nedge = by ? s->at(s->L.nedge) : nullptr;
    }
    // the tile list: block tiles of the other domains (phi stage and update),
    // block tiles of the phi-summing domains (phi stage: merge), tiles of the
    // phi-summing update (whole rows of one plane)
    const int threads = int(b->block.x * b->block.y * b->block.z);
    bool row = true;
    auto push = [&](const mplb::BatchTile &tl) {
        if ((long long)b->tiles.size() >= b->max_tiles) return false;
        b->tiles.push_back(tl);
        return true;
    };
    int seg[3] = {0, 0, 0};
    int wstart[mplb::NPHI_GROUPS] = {}, wcount[mplb::NPHI_GROUPS] = {};  // phi-summing tiles by row length
    for (int pass = 0; pass < 2 + mplb::NPHI_GROUPS; ++pass) {
        const size_t before = b->tiles.size();
        for (int i = 0; i < b->capacity; ++i) {
            const mplb_solver *s = b->slot[i];
            if (!s || b->solo[i]) continue;
            const int nx = s->prm.n[0], ny = s->prm.n[1], nz = s->prm.n[2];
            const int nby = b->doms[i].nphi_by;
            if (pass >= 2) {
                // one group per row length (nphi_group)
                if (!nby || nx != mplb::nphi_group_width(pass - 2)) continue;
                for (int z = 0; z < nz; ++z)
                    for (int y0 = 0; y0 < ny; y0 += nby)
                        if (!push(mplb::BatchTile{i, 0, y0, z, z + 1, nx}))
                            return fail(MPLB_ENOMEM, "batch tile list is full");
                continue;
            }
            if ((pass == 0) != (nby == 0)) continue;
            // tile width: the domain's row rounded up to a power of two, at
            // least 64 where the row form can apply (x periodic), at most the
            // block's width; the rest of the block's threads cover further rows
            int w = 1;
            while (w < nx) w <<= 1;
            const bool xper = b->doms[i].g.bcx == mplb::BC_PER;
            if (xper && w < 64) w = 64;
            if (w > int(b->block.x)) w = int(b->block.x);
            if (w > threads) w = threads;
            const int rows = threads / w;
            row = row && mplb::row_form_ok(b->dim, b->doms[i].g, dim3(w, rows, 1));
            for (int z0 = 0; z0 < nz; ++z0)
                for (int y0 = 0; y0 < ny; y0 += rows)
                    for (int x0 = 0; x0 < nx; x0 += w)
                        if (!push(mplb::BatchTile{i, x0, y0, z0, z0 + 1, w}))
                            return fail(MPLB_ENOMEM, "batch tile list is full");
        }
        if (pass < 2) {
            seg[pass] = int(b->tiles.size() - before);
        } else {
            wstart[pass - 2] = int(before);
            wcount[pass - 2] = int(b->tiles.size() - before);
            seg[2] += wcount[pass - 2];
        }
    }
    b->ntiles_host = seg[0];
    b->ntiles_phi_host = seg[0] + seg[1];
    b->ntiles_nphi_host = seg[2];
    {
        // one block per tile, hardware-scheduled; the launch sizes move in
        // buckets of 4096 blocks so that a captured graph survives most
        // attach / detach events (surplus blocks find no tile and exit)
        const int bucket = 4096;
        auto bucketed = [&](int n, int empty) { return n ? (n + bucket - 1) / bucket * bucket : empty; };
        constexpr int NG = 2 + mplb::NPHI_GROUPS;
        int grid[NG] = {bucketed(b->ntiles_phi_host, bucket), bucketed(b->ntiles_host, bucket)};
        for (int k = 0; k < mplb::NPHI_GROUPS; ++k) grid[2 + k] = bucketed(wcount[k], 0);
        for (int k = 0; k < NG; ++k)
            if (grid[k] != b->grid[k]) drop_graph(b);
        for (int k = 0; k < NG; ++k) b->grid[k] = grid[k];
    }
    if (row != b->row) drop_graph(b);  // a captured graph holds the other kernel
    b->row = row;
    HIPCHK(hipStreamSynchronize(b->stream));
    HIPCHK(hipMemcpyAsync(b->d_doms, b->doms.data(), sizeof(mplb::BatchDom) * b->capacity,
                          hipMemcpyHostToDevice, b->stream));
    if (!b->tiles.empty())
        HIPCHK(hipMemcpyAsync(b->d_tiles, b->tiles.data(), sizeof(mplb::BatchTile) * b->tiles.size(),
                              hipMemcpyHostToDevice, b->stream));
    b->counts[0] = b->ntiles_host;
    b->counts[1] = b->ntiles_phi_host;
    for (int k = 0; k < mplb::NPHI_GROUPS; ++k) {
        b->counts[2 + 2 * k] = wstart[k];
        b->counts[3 + 2 * k] = wcount[k];
    }
    HIPCHK(hipMemcpyAsync(b->d_ntiles, b->counts, sizeof(b->counts), hipMemcpyHostToDevice,
                          b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    return MPLB_OK;
}

}  // namespace

extern "C" {

size_t mplb_batch_table_bytes(int32_t capacity, int64_t max_tiles)
{
    if (capacity < 1 || max_tiles < 1) return 0;
    size_t a, b, c, d, e;
    return table_layout(capacity, max_tiles, &a, &b, &c, &d, &e);
}

int mplb_batch_create(int32_t dim, int32_t storage, int32_t capacity, int64_t max_tiles,
                      void *dev_table, size_t table_bytes, void *hip_stream, mplb_batch **out)
{
    if (!out) return fail(MPLB_EINVAL, "out is NULL");
    *out = nullptr;
    if (dim != 2 && dim != 3) return fail(MPLB_EINVAL, "dim must be 2 or 3");
    if (storage < MPLB_STORE_FP64 || storage > MPLB_STORE_FP16S_ALL)
        return fail(MPLB_EINVAL, "unknown storage format");
    if (capacity < 1 || max_tiles < 1 || max_tiles > 0x7fffffff)
        return fail(MPLB_EINVAL, "capacity and max_tiles must be >= 1");
    if (!dev_table || reinterpret_cast<uintptr_t>(dev_table) % ALIGN)
        return fail(MPLB_EINVAL, "table memory must be non-NULL and 256-byte aligned");
    if (!hip_stream)
        return fail(MPLB_EINVAL, "a batch needs its own stream (graphs cannot capture the null stream)");
    size_t od, ot, on, ob, os;
    const size_t need = table_layout(capacity, max_tiles, &od, &ot, &on, &ob, &os);
    if (table_bytes < need) return fail(MPLB_ENOMEM, "batch table memory too small");
    mplb_batch *b = new (std::nothrow) mplb_batch();
    if (!b) return fail(MPLB_ENOMEM, "host allocation failed");
    char *base = static_cast<char *>(dev_table);
    b->dim = dim;
    b->storage = storage;
    b->collision = MPLB_COLL_CUMULANT;
    b->capacity = capacity;
    b->max_tiles = max_tiles;
    b->stream = static_cast<hipStream_t>(hip_stream);
    b->d_doms = reinterpret_cast<mplb::BatchDom *>(base + od);
    b->d_tiles = reinterpret_cast<mplb::BatchTile *>(base + ot);
    b->d_ntiles = reinterpret_cast<int *>(base + on);
    b->d_tbase = reinterpret_cast<long long *>(base + ob);
    b->d_status = reinterpret_cast<int *>(base + os);
    b->slot.assign(capacity, nullptr);
    b->doms.assign(capacity, mplb::BatchDom{});
    b->solo.assign(capacity, 0);
    b->start.assign(capacity, 0);
    b->solo_min = 1ll << 20;
    b->nshared = 0;
    // a second stream at the default priority for the batched launches
    if (hipStreamCreate(&b->side) != hipSuccess) {
        delete b;
        return fail(MPLB_EDEVICE, "hipStreamCreate failed");
    }
    if (hipEventCreateWithFlags(&b->ev_main, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_side, hipEventDisableTiming) != hipSuccess) {
        (void)hipStreamDestroy(b->side);
        delete b;
        return fail(MPLB_EDEVICE, "hipEventCreate failed");
    }
    b->ntiles_host = b->ntiles_phi_host = b->ntiles_nphi_host = 0;
    // one bucket: an empty batch launches blocks that find no tile
    b->grid[0] = b->grid[1] = 4096;
    for (int k = 2; k < 2 + mplb::NPHI_GROUPS; ++k) b->grid[k] = 0;
    b->block = dim3(64, 4, 1);
    b->chunk = 16;
    b->t = 0;
    b->have_graph = false;
    b->row = true;
    int rc = upload_tables(b);
    if (rc == MPLB_OK && mplb::launch_fill_i32(b->d_status, capacity, 0, b->stream) != hipSuccess)
        rc = fail(MPLB_EDEVICE, "clearing the batch status flags failed");
    if (rc == MPLB_OK && hipStreamSynchronize(b->stream) != hipSuccess)
        rc = fail(MPLB_EDEVICE, "hipStreamSynchronize failed");
    if (rc != MPLB_OK) {
        (void)hipEventDestroy(b->ev_main);
        (void)hipEventDestroy(b->ev_side);
        (void)hipStreamDestroy(b->side);
        delete b;
        return rc;
    }
    *out = b;
    return MPLB_OK;
}

int mplb_batch_set_block(mplb_batch *b, int32_t bx, int32_t by, int32_t bz)
{
    if (!b) return fail(MPLB_EINVAL, "batch is NULL");
    if (bx < 1 || by < 1 || bz < 1 || (long long)bx * by * bz > 256)
        return fail(MPLB_EINVAL, "block must have between 1 and 256 threads");
    if (b->dim == 2 && bz != 1) return fail(MPLB_EINVAL, "bz must be 1 in 2-D");
    b->block = dim3(bx, by, bz);
    drop_graph(b);
    return upload_tables(b);
}

int mplb_batch_set_graph_chunk(mplb_batch *b, int32_t chunk)
{
    if (!b) return fail(MPLB_EINVAL, "batch is NULL");
    if (chunk < 0 || chunk > 4096) return fail(MPLB_EINVAL, "chunk must be in [0, 4096]");
    b->chunk = chunk;
    drop_graph(b);
    return MPLB_OK;
}

int mplb_batch_attach(mplb_batch *b, mplb_solver *s, int64_t nsteps, int32_t *slot)
{
    if (!b || !s || !slot) return fail(MPLB_EINVAL, "batch, solver and slot are required");
    if (nsteps < 0) return fail(MPLB_EINVAL, "nsteps must be >= 0");
    if (s->prm.dim != b->dim || s->prm.storage != b->storage)
        return fail(MPLB_EINVAL, "solver dimension/storage differ from the batch's");
    bool empty = true;
    for (auto *o : b->slot) empty = empty && !o;
    // operator code: flow collision (bit 0), first-order phase-field equilibrium (bit 1)
    const int code = s->prm.collision | (s->prm.cac_edf << 1);
    if (empty) {
        if (b->collision != code) drop_graph(b);
        b->collision = code;
    } else if (code != b->collision) {
        return fail(MPLB_EINVAL,
                    "solvers of one batch must share the collision operator and phase-field equilibrium");
    }
    if (s->stream != b->stream) return fail(MPLB_EINVAL, "solver and batch streams differ");
    if (!s->ready) return fail(MPLB_ESTATE, "solver is not initialised");
    if (s->attached) return fail(MPLB_ESTATE, "solver is already attached");
    int k = -1;
    for (int i = 0; i < b->capacity; ++i)
        if (!b->slot[i]) {
            k = i;
            break;
        }
    if (k < 0) return fail(MPLB_ENOMEM, "no free batch slot");
    mplb::BatchDom d{};
    const mplb::Ctx c = s->ctx(0);
    d.g = c.g;
    d.ph = s->ph;
    for (int j = 0; j < 2; ++j) {
        d.F[j] = s->F(j);
        d.G[j] = s->G(j);
        d.frest[j] = static_cast<float *>(s->at(s->L.frest[j]));
        d.grest[j] = static_cast<float *>(s->at(s->L.grest[j]));
        d.phiu[j] = s->at(s->L.phiu[j]);
    }
    // the domain's first batch step is b->t: history from there if it has one
    d.hist_from = s->hist ? b->t : b->t + 1;
    d.phi = s->base + s->L.phi;
    d.ref = static_cast<unsigned *>(s->at(s->L.ref));
    // the phi-summing update: upload_tables sets nphi_by and the pointers; a
    // solver whose last update left partial sums merges them at its first
    // batch step, as its own next step would
    d.nphi_by = (b->dim == 3 && s->use_nphi(s->ctx(s->cur))) ? s->next_phi().by : 0;
    d.nphi_from = s->nphi_valid ? b->t : b->t + 1;
    // input buffer at batch step t is (t - first) & 1; at t = b->t it is s->cur
    d.first = b->t - s->cur;
    d.last = b->t + nsteps;
    b->slot[k] = s;
    b->doms[k] = d;
    b->solo[k] = s->L.N >= b->solo_min ? 1 : 0;
    b->start[k] = b->t;
    s->attached = true;
    HIPCHK(mplb::launch_fill_i32(b->d_status + k, 1, 0, b->stream));
    const int rc = upload_tables(b);
    if (rc != MPLB_OK) {
        b->slot[k] = nullptr;
        b->doms[k] = mplb::BatchDom{};
        b->solo[k] = 0;
        s->attached = false;
        (void)upload_tables(b);
        return rc;
    }
    *slot = k;
    return MPLB_OK;
}

int mplb_batch_detach(mplb_batch *b, int32_t slot)
{
    if (!b || slot < 0 || slot >= b->capacity || !b->slot[slot])
        return fail(MPLB_EINVAL, "no solver in that slot");
    b->slot[slot]->attached = false;
    b->slot[slot] = nullptr;
    b->doms[slot] = mplb::BatchDom{};
    b->solo[slot] = 0;
    return upload_tables(b);
}

int mplb_batch_remaining(const mplb_batch *b, int32_t slot, int64_t *remaining)
{
    if (!b || !remaining || slot < 0 || slot >= b->capacity || !b->slot[slot])
        return fail(MPLB_EINVAL, "no solver in that slot");
    const long long r = b->doms[slot].last - b->t;
    *remaining = r > 0 ? r : 0;
    return MPLB_OK;
}

int64_t mplb_batch_steps_done(const mplb_batch *b) { return b ? b->t : -1; }

int mplb_batch_status(mplb_batch *b, int32_t *status)
{
    if (!b || !status) return fail(MPLB_EINVAL, "batch and status are required");
    std::vector<int> flags(b->capacity);
    HIPCHK(hipMemcpyAsync(flags.data(), b->d_status, sizeof(int) * b->capacity,
                          hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    bool closed = false;
    for (int i = 0; i < b->capacity; ++i) {
        if (!b->slot[i]) {
            status[i] = MPLB_ESTATE;
            continue;
        }
        status[i] = flags[i] ? MPLB_EUNSTABLE : MPLB_OK;
        if (flags[i] && b->doms[i].last > b->t) {
            // retire: the slot takes no further batch steps
            b->doms[i].last = b->t;
            closed = true;
        }
    }
    return closed ? upload_tables(b) : MPLB_OK;
}

int mplb_batch_step(mplb_batch *b, int64_t nsteps)
{
    if (!b) return fail(MPLB_EINVAL, "batch is NULL");
    if (nsteps < 0) return fail(MPLB_EINVAL, "nsteps must be >= 0");
    if (nsteps == 0) return MPLB_OK;
    const long long t0 = b->t;
    // the batched launches follow the work queued on the solvers' stream
    HIPCHK(hipEventRecord(b->ev_main, b->stream));
    HIPCHK(hipStreamWaitEvent(b->side, b->ev_main, 0));
    long long done = 0;
    while (b->nshared > 0 && done < nsteps) {
        const long long left = nsteps - done;
        HIPCHK(mplb::launch_set_i64(b->d_tbase, b->t, b->side));
        if (b->chunk > 0 && left >= b->chunk) {
            if (!b->have_graph) {
                hipGraph_t graph = nullptr;
                HIPCHK(hipStreamBeginCapture(b->side, hipStreamCaptureModeThreadLocal));
                hipError_t e = hipSuccess;
                for (int k = 0; k < b->chunk && e == hipSuccess; ++k)
                    e = mplb::launch_batch_step(b->dim, b->storage, b->collision, b->row,
                                                b->d_doms, b->d_tiles, b->d_ntiles, b->d_tbase, k,
                                                b->block, b->grid, b->d_status, b->side);
                // always end the capture, so that a failure leaves the stream usable
                const hipError_t e2 = hipStreamEndCapture(b->side, &graph);
                if (e != hipSuccess || e2 != hipSuccess) {
                    if (graph) (void)hipGraphDestroy(graph);
                    return fail(MPLB_EDEVICE, std::string("graph capture: ") +
                                                  hipGetErrorString(e != hipSuccess ? e : e2));
                }
                e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
                (void)hipGraphDestroy(graph);
                if (e != hipSuccess)
                    return fail(MPLB_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
                b->have_graph = true;
            }
            HIPCHK(hipGraphLaunch(b->exec, b->side));
            b->t += b->chunk;
            done += b->chunk;
        } else {
            HIPCHK(mplb::launch_batch_step(b->dim, b->storage, b->collision, b->row, b->d_doms,
                                           b->d_tiles, b->d_ntiles, b->d_tbase, 0, b->block,
                                           b->grid, b->d_status, b->side));
            b->t += 1;
            done += 1;
        }
    }
    b->t = t0 + nsteps;
    // domains that step with their own kernels (runs of steps as their step
    // graphs), on the solvers' stream while the batched launches run on the
    // side stream; their phi is checked for non-finite values before every
    // graph run and every chunk of direct steps
    const int check = b->chunk > 0 ? b->chunk : 16;
    for (int i = 0; i < b->capacity; ++i) {
        mplb_solver *s = b->slot[i];
        if (!s || !b->solo[i]) continue;
        const long long lo = t0 > b->start[i] ? t0 : b->start[i];
        const long long hi = b->t < b->doms[i].last ? b->t : b->doms[i].last;
        for (long long k = lo; k < hi;) {
            const mplb::Ctx c = s->ctx(s->cur);
            const bool steady = s->hist && (!s->use_nphi(c) || s->nphi_valid);
            if (steady && hi - k >= GRAPH_STEPS) {
                // a run of steps as the solver's step graph, its phi checked first
                HIPCHK(mplb::launch_flag_nonfinite(c, b->d_status + i));
                const int rc = replay_steps(s);
                if (rc != MPLB_OK) return rc;
                s->steps += GRAPH_STEPS;
                k += GRAPH_STEPS;
                continue;
            }
            HIPCHK(s->launch_phi_stage(c));
            if ((k - lo) % check == 0) HIPCHK(mplb::launch_flag_nonfinite(c, b->d_status + i));
            HIPCHK(s->launch_update_stage(c));
            s->cur ^= 1;
            s->steps++;
            s->hist = true;
            ++k;
        }
    }
    HIPCHK(hipEventRecord(b->ev_side, b->side));
    HIPCHK(hipStreamWaitEvent(b->stream, b->ev_side, 0));
    // host bookkeeping of the shared domains: each advanced by the overlap of
    // its window with [t0, t); windows open at or before t0
    for (int i = 0; i < b->capacity; ++i) {
        mplb_solver *s = b->slot[i];
        if (!s || b->solo[i]) continue;
        const long long lo = t0;
        const long long hi = b->t < b->doms[i].last ? b->t : b->doms[i].last;
        const long long adv = hi > lo ? hi - lo : 0;
        s->steps += adv;
        s->cur = int((s->cur + adv) & 1);
        if (adv > 0) {
            s->hist = true;
            // the batched update left partial sums of phi if it summed them
            s->nphi_valid = b->doms[i].nphi_by > 0;
        }
    }
    return MPLB_OK;
}

int mplb_batch_set_solo_cells(mplb_batch *b, int64_t min_cells)
{
    if (!b) return fail(MPLB_EINVAL, "batch is NULL");
    if (min_cells < 0) return fail(MPLB_EINVAL, "min_cells must be >= 0");
    b->solo_min = min_cells;
    return MPLB_OK;
}

int mplb_batch_is_solo(const mplb_batch *b, int32_t slot)
{
    if (!b || slot < 0 || slot >= b->capacity || !b->slot[slot])
        return fail(MPLB_EINVAL, "no solver in that slot");
    return b->solo[slot] ? 1 : 0;
}

int mplb_batch_tune_block(mplb_batch *b, int32_t steps, const int32_t *candidates, int32_t ncand,
                          int32_t best[3], double *best_ms_per_step)
{
    static const int32_t builtin3[] = {64, 4, 1, 64, 2, 2, 128, 2, 1, 128, 1, 2, 256, 1, 1,
                                       64, 1, 4, 32, 8, 1, 32, 4, 2};
    static const int32_t builtin2[] = {64, 4, 1, 128, 2, 1, 256, 1, 1, 64, 2, 1, 32, 8, 1,
                                       16, 16, 1};
    if (!b || !best || !best_ms_per_step) return fail(MPLB_EINVAL, "batch and outputs are required");
    if (steps < 1) return fail(MPLB_EINVAL, "steps must be >= 1");
    bool any = false;
    for (auto *s : b->slot) any = any || s;
    if (!any) return fail(MPLB_EINVAL, "no attached domain to time");
    if (!candidates) {
        candidates = b->dim == 3 ? builtin3 : builtin2;
        ncand = b->dim == 3 ? int32_t(sizeof(builtin3) / 12) : int32_t(sizeof(builtin2) / 12);
    }
    const dim3 keep = b->block;
    const int keep_chunk = b->chunk;
    b->chunk = 0;  // direct launches while tuning: every candidate pays the same launch cost
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(MPLB_EDEVICE, "hipEventCreate failed");
    }
    double best_ms = 1e300;
    int rc = MPLB_OK;
    for (int i = 0; i < ncand && rc == MPLB_OK; ++i) {
        const int32_t *c = candidates + 3 * i;
        if (b->dim == 2 && c[2] != 1) continue;
        if (mplb_batch_set_block(b, c[0], c[1], c[2]) != MPLB_OK) continue;
        rc = mplb_batch_step(b, 1);
        if (rc != MPLB_OK) break;
        if (hipEventRecord(e0, b->stream) != hipSuccess) { rc = fail(MPLB_EDEVICE, "event"); break; }
        rc = mplb_batch_step(b, steps);
        if (rc != MPLB_OK) break;
        float ms = 0;
        if (hipEventRecord(e1, b->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = fail(MPLB_EDEVICE, "event timing failed");
            break;
        }
        if (ms / steps < best_ms) {
            best_ms = ms / steps;
            best[0] = c[0];
            best[1] = c[1];
            best[2] = c[2];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->chunk = keep_chunk;
    if (rc == MPLB_OK && best_ms == 1e300) rc = fail(MPLB_EINVAL, "no valid candidate block shape");
    const int rs = rc == MPLB_OK ? mplb_batch_set_block(b, best[0], best[1], best[2])
                                 : mplb_batch_set_block(b, keep.x, keep.y, keep.z);
    if (rc != MPLB_OK) return rc;
    if (rs != MPLB_OK) return rs;
    *best_ms_per_step = best_ms;
    return MPLB_OK;
}

void mplb_batch_destroy(mplb_batch *b)
{
    if (!b) return;
    for (auto *s : b->slot)
        if (s) s->attached = false;
    (void)hipStreamSynchronize(b->side);
    drop_graph(b);
    (void)hipEventDestroy(b->ev_main);
    (void)hipEventDestroy(b->ev_side);
    (void)hipStreamDestroy(b->side);
    delete b;
}

}  // extern "C"
