// mc_api.hip -- C ABI of libmc.so: context, data upload, the host side of the
// event loop and tally statistics.  Declarations and argument contracts are in
// include/mc.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mc.h"
#include "mc_device.h"
#include "mc_internal.h"
#include "mc_physics.h"

using namespace mc;

namespace {

constexpr uint64_t kDefaultInFlight = 1ull << 20;
constexpr uint64_t kDefaultSortMin = 16384;
constexpr int64_t kDefaultMaxEvents = 100000;
constexpr int64_t kDefaultTailParticles = 32768;

struct Buffers {
    std::vector<void *> ptrs;
    void release()
    {
        for (void *p : ptrs) (void)hipFree(p);
        ptrs.clear();
    }
};

}  // namespace

struct mc_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;

    // materials
    bool have_mat = false;
    Buffers mat_bufs;
    XsDev xs{};
    int32_t n_nuc = 0, n_mat = 0;
    std::vector<int32_t> mat_len;
    uint32_t n_keys = 0;  // n_mat * M sort keys

    // geometry and tallies
    bool have_geom = false;
    Buffers geom_bufs;
    GeomDev geom{};
    int32_t n_bins = 0;
    double *S1[3] = {nullptr, nullptr, nullptr}, *S2[3] = {nullptr, nullptr, nullptr};
    uint64_t n_batches = 0, histories = 0;

    // particle bank and per-workgroup tally rows
    Buffers bank_bufs;
    BankDev bank{};
    SortBufs bank_sort{};
    TallyDev tal{};
    double *partial = nullptr;
    uint32_t cap = 0;
    int32_t bank_bins = -1;

    // loop bookkeeping
    Buffers misc_bufs;
    Counters *ctr = nullptr;             // device, ring of 2
    Counters *ctr_host = nullptr;        // pinned host copy
    unsigned long long *dstat = nullptr; // device: [0] nuclide lookups, [1] lost

    // scratch of the stand-alone lookup / sort entry points
    Buffers scratch_bufs;
    size_t scratch_n = 0;
    uint32_t *s_perm = nullptr, *s_keys = nullptr;
    int32_t *s_mat = nullptr;
    SortBufs s_sort{};

    std::vector<hipEvent_t> ev_a, ev_b;
    hipEvent_t ev_batch0 = nullptr, ev_batch1 = nullptr;
    mc_stats stats{};
    bool timing = false;  // time the stand-alone lookups (mc_set_timing)
    mc_tuning tune{};      // launch shapes (0 = default)
};

static int lookup_ilp(const mc_ctx *ctx) { return ctx->tune.lookup_ilp ? ctx->tune.lookup_ilp : DEFAULT_LOOKUP_ILP; }
static int64_t tail_particles(const mc_ctx *ctx)
{
    return ctx->tune.tail_particles == 0 ? kDefaultTailParticles : (int64_t)ctx->tune.tail_particles;
}

static int fail(mc_ctx *c, int code, const std::string &msg)
{
    if (c) c->err = msg;
    return code;
}

#define HIPCHK(call)                                                                         \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(ctx, MC_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));    \
    } while (0)

template <class T>
static int dalloc(mc_ctx *ctx, Buffers &b, T **p, size_t count)
{
    *p = nullptr;
    if (count == 0) count = 1;
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, count * sizeof(T));
    if (e != hipSuccess) return fail(ctx, MC_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    b.ptrs.push_back(q);
    *p = static_cast<T *>(q);
    return MC_OK;
}

template <class T>
static int upload(mc_ctx *ctx, Buffers &b, T **p, const T *host, size_t count)
{
    int rc = dalloc(ctx, b, p, count);
    if (rc) return rc;
    if (count) HIPCHK(hipMemcpy(*p, host, count * sizeof(T), hipMemcpyHostToDevice));
    return MC_OK;
}

// i(E) = max{j : grid[j] <= E} clamped to [0, N-2]
static int32_t host_grid_index(const double *grid, int32_t n, double e)
{
    const double *ub = std::upper_bound(grid, grid + n, e);
    int32_t i = (int32_t)(ub - grid) - 1;
    return std::min(std::max(i, 0), n - 2);
}

static void build_bounds(const double *E, int32_t N, double emin, double emax, int32_t M, int32_t *lo)
{
    const double delta = std::log(emax / emin) / (double)M;
    for (int32_t b = 0; b < M; ++b) lo[b] = host_grid_index(E, N, emin * std::exp((double)b * delta));
    lo[M] = N - 2;
}

extern "C" {

const char *mc_version(void) { return "mc355 0.1 (gfx950)"; }

int mc_create(mc_ctx **out, int device, void *hip_stream)
{
    if (!out) return MC_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0 || device < 0 || device >= n) return MC_ENODEV;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return MC_EHIP;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return MC_ENODEV;
    if (hipSetDevice(device) != hipSuccess) return MC_EHIP;
    mc_ctx *ctx = new (std::nothrow) mc_ctx();
    if (!ctx) return MC_ENOMEM;
    ctx->device = device;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    int rc = dalloc(ctx, ctx->misc_bufs, &ctx->ctr, 2);
    if (!rc) rc = dalloc(ctx, ctx->misc_bufs, &ctx->dstat, 4);
    if (!rc && hipHostMalloc((void **)&ctx->ctr_host, 2 * sizeof(Counters), hipHostMallocDefault) != hipSuccess)
        rc = MC_ENOMEM;
    if (!rc && (hipEventCreate(&ctx->ev_batch0) != hipSuccess || hipEventCreate(&ctx->ev_batch1) != hipSuccess))
        rc = MC_EHIP;
    if (rc) {
        mc_destroy(ctx);
        return rc;
    }
    *out = ctx;
    return MC_OK;
}

void mc_destroy(mc_ctx *ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    ctx->mat_bufs.release();
    ctx->geom_bufs.release();
    ctx->bank_bufs.release();
    ctx->misc_bufs.release();
    ctx->scratch_bufs.release();
    if (ctx->ctr_host) (void)hipHostFree(ctx->ctr_host);
    for (hipEvent_t e : ctx->ev_a) (void)hipEventDestroy(e);
    for (hipEvent_t e : ctx->ev_b) (void)hipEventDestroy(e);
    if (ctx->ev_batch0) (void)hipEventDestroy(ctx->ev_batch0);
    if (ctx->ev_batch1) (void)hipEventDestroy(ctx->ev_batch1);
    delete ctx;
}

const char *mc_last_error(const mc_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int mc_set_stream(mc_ctx *ctx, void *hip_stream)
{
    if (!ctx) return MC_EINVAL;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    return MC_OK;
}

int mc_hash_bounds(const double *E, int32_t N, double emin, double emax, int32_t M, int32_t *lo)
{
    if (!E || !lo || N < 2 || M < 1 || !(emin > 0.0) || !(emax > emin)) return MC_EINVAL;
    build_bounds(E, N, emin, emax, M, lo);
    return MC_OK;
}

int mc_init_materials(mc_ctx *ctx, int32_t n_nuc, const int32_t *grid_len, const double *const *E,
                      const double *const *sig_c, const double *const *sig_s, const double *awr,
                      int32_t n_mat, const int32_t *mat_len, const int32_t *mat_nuc,
                      const double *mat_dens, int32_t n_hash_bins)
{
    if (!ctx) return MC_EINVAL;
    if (n_nuc < 1 || !grid_len || !E || !sig_c || !sig_s || !awr || n_mat < 1 || !mat_len || !mat_nuc ||
        !mat_dens || n_hash_bins < 1)
        return fail(ctx, MC_EINVAL, "mc_init_materials: missing array or non-positive count");
    HIPCHK(hipSetDevice(ctx->device));
    // validate nuclides
    uint64_t total = 0;
    double emin = INFINITY, emax = 0.0;
    for (int32_t k = 0; k < n_nuc; ++k) {
        const int32_t n = grid_len[k];
        if (n < 2 || !E[k] || !sig_c[k] || !sig_s[k])
            return fail(ctx, MC_EINVAL, "nuclide " + std::to_string(k) + ": grid shorter than 2 points");
        if (!(awr[k] > 0.0) || !std::isfinite(awr[k]))
            return fail(ctx, MC_EINVAL, "nuclide " + std::to_string(k) + ": mass ratio must be > 0");
        for (int32_t j = 0; j < n; ++j) {
            if (!std::isfinite(E[k][j]) || !(E[k][j] > 0.0))
                return fail(ctx, MC_EINVAL, "nuclide " + std::to_string(k) + ": energy not finite and > 0");
            if (j && !(E[k][j] > E[k][j - 1]))
                return fail(ctx, MC_EINVAL,
                            "nuclide " + std::to_string(k) + ": grid not strictly increasing at point " +
                                std::to_string(j));
            if (!(sig_c[k][j] >= 0.0) || !(sig_s[k][j] >= 0.0) || !std::isfinite(sig_c[k][j]) ||
                !std::isfinite(sig_s[k][j]))
                return fail(ctx, MC_EINVAL, "nuclide " + std::to_string(k) + ": cross section < 0 or not finite");
        }
        total += (uint64_t)n;
        emin = std::min(emin, E[k][0]);
        emax = std::max(emax, E[k][n - 1]);
    }
    if (total >= (1ull << 32)) return fail(ctx, MC_EINVAL, "more than 2^32 grid points in total");
    uint64_t n_entries = 0;
    for (int32_t m = 0; m < n_mat; ++m) {
        if (mat_len[m] < 1) return fail(ctx, MC_EINVAL, "material " + std::to_string(m) + " has no nuclides");
        for (int32_t q = 0; q < mat_len[m]; ++q) {
            const int32_t k = mat_nuc[n_entries + q];
            const double d = mat_dens[n_entries + q];
            if (k < 0 || k >= n_nuc)
                return fail(ctx, MC_EINVAL, "material " + std::to_string(m) + ": unknown nuclide id " +
                                                std::to_string(k));
            if (!(d > 0.0) || !std::isfinite(d))
                return fail(ctx, MC_EINVAL, "material " + std::to_string(m) + ": density must be > 0");
        }
        n_entries += (uint64_t)mat_len[m];
    }
    if ((uint64_t)n_mat * (uint64_t)n_hash_bins >= (1ull << 32))
        return fail(ctx, MC_EINVAL, "n_mat * n_hash_bins must stay below 2^32");

    // host tables
    std::vector<double> Eg(total);
    std::vector<double> xs(2 * total);
    std::vector<uint32_t> off(n_nuc);
    uint64_t p = 0;
    for (int32_t k = 0; k < n_nuc; ++k) {
        off[k] = (uint32_t)p;
        for (int32_t j = 0; j < grid_len[k]; ++j, ++p) {
            Eg[p] = E[k][j];
            xs[2 * p] = sig_c[k][j];
            xs[2 * p + 1] = sig_s[k][j];
        }
    }
    const int32_t M = n_hash_bins;
    std::vector<int32_t> lo((size_t)n_nuc * (M + 1));
    for (int32_t k = 0; k < n_nuc; ++k) build_bounds(E[k], grid_len[k], emin, emax, M, &lo[(size_t)k * (M + 1)]);
    std::vector<int32_t> moff(n_mat + 1);
    std::vector<MatNuc> mnuc(n_entries);
    std::vector<uint64_t> hoff(n_mat);
    uint64_t hash_words = 0;
    moff[0] = 0;
    for (int32_t m = 0; m < n_mat; ++m) {
        moff[m + 1] = moff[m] + mat_len[m];
        hoff[m] = hash_words;
        hash_words += (uint64_t)(M + 1) * (uint64_t)mat_len[m];
    }
    std::vector<uint32_t> hash(hash_words);
    for (int32_t m = 0; m < n_mat; ++m) {
        const int32_t nk = mat_len[m];
        for (int32_t q = 0; q < nk; ++q) {
            const int32_t k = mat_nuc[moff[m] + q];
            mnuc[moff[m] + q] = MatNuc{off[k], (uint32_t)grid_len[k], mat_dens[moff[m] + q]};
            for (int32_t b = 0; b <= M; ++b)
                hash[hoff[m] + (uint64_t)b * nk + q] = (uint32_t)lo[(size_t)k * (M + 1) + b];
        }
    }

    HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->mat_bufs.release();
    ctx->have_mat = false;
    ctx->have_geom = false;
    XsDev x{};
    double *d_Eg, *d_awr;
    double2 *d_xs;
    int32_t *d_moff, *d_mnucid;
    MatNuc *d_mnuc;
    uint32_t *d_hash;
    uint64_t *d_hoff;
    int rc = upload(ctx, ctx->mat_bufs, &d_Eg, Eg.data(), Eg.size());
    if (!rc) rc = upload(ctx, ctx->mat_bufs, &d_xs, reinterpret_cast<const double2 *>(xs.data()), total);
    if (!rc) rc = upload(ctx, ctx->mat_bufs, &d_awr, awr, (size_t)n_nuc);
    if (!rc) rc = upload(ctx, ctx->mat_bufs, &d_moff, moff.data(), moff.size());
    if (!rc) rc = upload(ctx, ctx->mat_bufs, &d_mnucid, mat_nuc, (size_t)n_entries);
    if (!rc) rc = upload(ctx, ctx->mat_bufs, &d_mnuc, mnuc.data(), mnuc.size());
    if (!rc) rc = upload(ctx, ctx->mat_bufs, &d_hash, hash.data(), hash.size());
    if (!rc) rc = upload(ctx, ctx->mat_bufs, &d_hoff, hoff.data(), hoff.size());
    ctx->n_keys = (uint32_t)((uint64_t)n_mat * (uint64_t)M);
    if (rc) {
        ctx->mat_bufs.release();
        return rc;
    }
    x.Eg = d_Eg;
    x.xs = d_xs;
    x.awr = d_awr;
    x.mat_off = d_moff;
    x.mat_nuc = d_mnucid;
    x.mnuc = d_mnuc;
    x.hash = d_hash;
    x.hash_off = d_hoff;
    x.n_mat = n_mat;
    x.M = M;
    x.ln_emin = std::log(emin);
    x.inv_delta = (double)M / std::log(emax / emin);
    ctx->xs = x;
    ctx->n_nuc = n_nuc;
    ctx->n_mat = n_mat;
    ctx->mat_len.assign(mat_len, mat_len + n_mat);
    ctx->have_mat = true;
    return MC_OK;
}

static int reset_tallies(mc_ctx *ctx)
{
    for (int t = 0; t < 3; ++t) {
        const size_t n = (t == 2) ? (size_t)N_GLOBAL : (size_t)ctx->n_bins;
        HIPCHK(launch_fill_f64(ctx->S1[t], n, 0.0, ctx->stream));
        HIPCHK(launch_fill_f64(ctx->S2[t], n, 0.0, ctx->stream));
    }
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->n_batches = 0;
    ctx->histories = 0;
    return MC_OK;
}

int mc_reset_tallies(mc_ctx *ctx)
{
    if (!ctx) return MC_EINVAL;
    if (!ctx->have_geom) return fail(ctx, MC_ESTATE, "no geometry");
    HIPCHK(hipSetDevice(ctx->device));
    return reset_tallies(ctx);
}

int mc_init_geometry(mc_ctx *ctx, const mc_geometry_desc *d)
{
    if (!ctx || !d) return MC_EINVAL;
    if (!ctx->have_mat) return fail(ctx, MC_ESTATE, "mc_init_geometry: materials first");
    HIPCHK(hipSetDevice(ctx->device));
    auto bad = [&](const std::string &m) { return fail(ctx, MC_EINVAL, "mc_init_geometry: " + m); };
    auto mat_ok = [&](int32_t m) { return m >= 0 && m < ctx->n_mat; };
    for (int f = 0; f < 6; ++f)
        if (d->bc[f] != MC_BC_REFLECT && d->bc[f] != MC_BC_VACUUM) return bad("unknown boundary condition");
    int32_t n_bins = 0;
    switch (d->kind) {
    case MC_GEOM_INFINITE:
        if (!mat_ok(d->material)) return bad("material id out of range");
        break;
    case MC_GEOM_LATTICE:
        if (d->nx < 1 || d->ny < 1 || !(d->pitch > 0.0) || !(d->radius > 0.0) || !(2.0 * d->radius < d->pitch) ||
            !(d->z1 > d->z0) || !d->pin_material)
            return bad("lattice needs nx, ny >= 1, 0 < 2 radius < pitch, z1 > z0 and pin_material");
        if ((int64_t)d->nx * d->ny > (1 << 30)) return bad("lattice too large");
        if (!mat_ok(d->moderator_material)) return bad("moderator material out of range");
        for (int64_t c = 0; c < (int64_t)d->nx * d->ny; ++c)
            if (d->pin_material[c] != -1 && !mat_ok(d->pin_material[c])) return bad("pin material out of range");
        break;
    case MC_GEOM_SLAB:
        if (d->n_layers < 1 || !d->x_edges || !d->layer_material) return bad("slab needs layers");
        for (int32_t l = 0; l < d->n_layers; ++l) {
            if (!(d->x_edges[l + 1] > d->x_edges[l])) return bad("slab edges must increase");
            if (!mat_ok(d->layer_material[l])) return bad("layer material out of range");
        }
        break;
    default:
        return bad("unknown geometry kind");
    }
    switch (d->tally_kind) {
    case MC_TALLY_ENERGY:
        if (d->n_energy_bins < 1 || !d->energy_edges) return bad("energy tally needs edges");
        for (int32_t b = 0; b < d->n_energy_bins; ++b)
            if (!(d->energy_edges[b + 1] > d->energy_edges[b])) return bad("energy edges must increase");
        n_bins = d->n_energy_bins;
        break;
    case MC_TALLY_PIN:
        if (d->kind != MC_GEOM_LATTICE) return bad("pin tally needs a lattice");
        n_bins = d->nx * d->ny;
        break;
    case MC_TALLY_MESH:
        for (int k = 0; k < 3; ++k)
            if (d->mesh_dims[k] < 1 || !(d->mesh_box[2 * k + 1] > d->mesh_box[2 * k])) return bad("bad mesh");
        if ((int64_t)d->mesh_dims[0] * d->mesh_dims[1] * d->mesh_dims[2] > (1 << 28)) return bad("mesh too large");
        n_bins = d->mesh_dims[0] * d->mesh_dims[1] * d->mesh_dims[2];
        break;
    case MC_TALLY_SLAB:
        if (d->kind != MC_GEOM_SLAB) return bad("slab tally needs a slab");
        n_bins = d->n_layers;
        break;
    default:
        return bad("unknown tally kind");
    }
    if (d->tally_kind != MC_TALLY_MESH && n_bins > MAX_LDS_BINS)
        return bad("more than 1024 bins needs a mesh tally");
    if (d->source_kind != MC_SRC_POINT && d->source_kind != MC_SRC_BOX && d->source_kind != MC_SRC_BEAM)
        return bad("unknown source kind");
    if (!(d->source_energy > 0.0) || !(d->energy_cutoff >= 0.0)) return bad("energies must be > 0");
    if (d->source_kind == MC_SRC_BEAM) {
        const double n2 = d->source_dir[0] * d->source_dir[0] + d->source_dir[1] * d->source_dir[1] +
                          d->source_dir[2] * d->source_dir[2];
        if (std::fabs(n2 - 1.0) > 1e-12) return bad("beam direction must be a unit vector");
    }

    HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->geom_bufs.release();
    ctx->have_geom = false;
    GeomDev g{};
    g.kind = d->kind;
    g.inf_mat = d->material;
    g.nx = d->nx;
    g.ny = d->ny;
    g.pitch = d->pitch;
    g.radius = d->radius;
    g.z0 = d->z0;
    g.z1 = d->z1;
    g.mod_mat = d->moderator_material;
    for (int f = 0; f < 6; ++f) g.bc[f] = d->bc[f];
    g.n_layers = d->n_layers;
    g.src_kind = d->source_kind;
    for (int k = 0; k < 3; ++k) {
        g.src_pos[k] = d->source_pos[k];
        g.src_dir[k] = d->source_dir[k];
    }
    for (int k = 0; k < 6; ++k) g.src_box[k] = d->source_box[k];
    g.src_E = d->source_energy;
    g.tally_kind = d->tally_kind;
    g.n_bins = n_bins;
    g.n_ebins = d->tally_kind == MC_TALLY_ENERGY ? d->n_energy_bins : 0;
    for (int k = 0; k < 3; ++k) {
        g.mesh_dims[k] = d->mesh_dims[k];
        g.mesh_lo[k] = d->mesh_box[2 * k];
        g.mesh_hi[k] = d->mesh_box[2 * k + 1];
    }
    g.e_cut = d->energy_cutoff;
    int rc = MC_OK;
    int32_t *pm;
    double *xe, *ee;
    int32_t *lm;
    const int32_t zero_i = 0;
    const double zero_d[2] = {0.0, 0.0};
    if (d->kind == MC_GEOM_LATTICE) rc = upload(ctx, ctx->geom_bufs, &pm, d->pin_material, (size_t)d->nx * d->ny);
    else rc = upload(ctx, ctx->geom_bufs, &pm, &zero_i, 1);
    if (!rc) {
        if (d->kind == MC_GEOM_SLAB) {
            rc = upload(ctx, ctx->geom_bufs, &xe, d->x_edges, (size_t)d->n_layers + 1);
            if (!rc) rc = upload(ctx, ctx->geom_bufs, &lm, d->layer_material, (size_t)d->n_layers);
        } else {
            rc = upload(ctx, ctx->geom_bufs, &xe, zero_d, 2);
            if (!rc) rc = upload(ctx, ctx->geom_bufs, &lm, &zero_i, 1);
        }
    }
    if (!rc) {
        if (d->tally_kind == MC_TALLY_ENERGY) rc = upload(ctx, ctx->geom_bufs, &ee, d->energy_edges, (size_t)n_bins + 1);
        else rc = upload(ctx, ctx->geom_bufs, &ee, zero_d, 2);
    }
    for (int t = 0; t < 3 && !rc; ++t) {
        const size_t n = (t == 2) ? (size_t)N_GLOBAL : (size_t)n_bins;
        rc = dalloc(ctx, ctx->geom_bufs, &ctx->S1[t], n);
        if (!rc) rc = dalloc(ctx, ctx->geom_bufs, &ctx->S2[t], n);
    }
    if (rc) {
        ctx->geom_bufs.release();
        return rc;
    }
    g.pin_mat = pm;
    g.x_edges = xe;
    g.layer_mat = lm;
    g.e_edges = ee;
    ctx->geom = g;
    ctx->n_bins = n_bins;
    ctx->have_geom = true;
    return reset_tallies(ctx);
}

// Radix-sort scratch for up to n items (chunk totals start at zero).
static int alloc_sort(mc_ctx *ctx, Buffers &B, SortBufs &sb, size_t n)
{
    int rc = dalloc(ctx, B, &sb.kA, n);
    if (!rc) rc = dalloc(ctx, B, &sb.kB, n);
    if (!rc) rc = dalloc(ctx, B, &sb.vA, n);
    if (!rc) rc = dalloc(ctx, B, &sb.vB, n);
    const size_t tiles = sort_tile_count(n), chunks = sort_chunk_count(n);
    if (!rc) rc = dalloc(ctx, B, &sb.tile_hist, tiles * 256);
    if (!rc) rc = dalloc(ctx, B, &sb.chunk_total, chunks * 256);
    if (!rc) rc = dalloc(ctx, B, &sb.chunk_off, chunks * 256);
    if (!rc) HIPCHK(hipMemset(sb.chunk_total, 0, chunks * 256 * sizeof(uint32_t)));
    return rc;
}

// Particle bank of capacity cap and the tally rows of its workgroups.
static int ensure_bank(mc_ctx *ctx, uint32_t cap)
{
    if (ctx->cap >= cap && ctx->bank_bins == ctx->n_bins && ctx->tal.n_bins == ctx->n_bins &&
        (ctx->geom.tally_kind == TALLY_MESH) == (ctx->tal.mesh_tl != nullptr))
        return MC_OK;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->bank_bufs.release();
    ctx->cap = 0;
    Buffers &B = ctx->bank_bufs;
    BankDev b{};
    b.C = cap;
    int rc = MC_OK;
    double **dd[] = {&b.x, &b.y, &b.z, &b.u, &b.v, &b.w, &b.E, &b.wt, &b.Sa, &b.Ss, &b.track};
    for (double **p : dd)
        if (!rc) rc = dalloc(ctx, B, p, cap);
    int32_t **ii[] = {&b.mat, &b.cell, &b.ncoll, &b.ncross};
    for (int32_t **p : ii)
        if (!rc) rc = dalloc(ctx, B, p, cap);
    uint8_t **bb[] = {&b.flags, &b.inside, &b.event};
    for (uint8_t **p : bb)
        if (!rc) rc = dalloc(ctx, B, p, cap);
    if (!rc) rc = dalloc(ctx, B, &b.pid, cap);
    uint32_t **uu[] = {&b.ndraw, &b.lineage, &b.A, &b.L, &b.Ls, &b.Lkey, &b.Qc, &b.Qx};
    for (uint32_t **p : uu)
        if (!rc) rc = dalloc(ctx, B, p, cap);
    const uint32_t n_tiles = (cap + TILE - 1) / TILE;
    if (!rc) rc = dalloc(ctx, B, &b.tile_cnt, (size_t)3 * n_tiles);
    TallyDev t{};
    t.n_bins = ctx->n_bins;
    t.rows = (int32_t)((cap + WG - 1) / WG);
    const bool mesh = ctx->geom.tally_kind == TALLY_MESH;
    const size_t row_bins = mesh ? 1 : (size_t)ctx->n_bins;
    if (!rc) rc = dalloc(ctx, B, &t.tl, (size_t)t.rows * row_bins);
    if (!rc) rc = dalloc(ctx, B, &t.coll, (size_t)t.rows * row_bins);
    if (!rc) rc = dalloc(ctx, B, &t.glob, (size_t)t.rows * N_GLOBAL);
    if (!rc && mesh) rc = dalloc(ctx, B, &t.mesh_tl, (size_t)ctx->n_bins);
    if (!rc && mesh) rc = dalloc(ctx, B, &t.mesh_coll, (size_t)ctx->n_bins);
    if (!rc) rc = dalloc(ctx, B, &ctx->partial, (size_t)64 * std::max<size_t>(ctx->n_bins, N_GLOBAL));
    SortBufs sb{};
    if (!rc) rc = alloc_sort(ctx, B, sb, cap);
    if (rc) {
        B.release();
        return rc;
    }
    ctx->bank = b;
    ctx->bank_sort = sb;
    ctx->tal = t;
    ctx->cap = cap;
    ctx->bank_bins = ctx->n_bins;
    return MC_OK;
}

static int ensure_scratch(mc_ctx *ctx, size_t n)
{
    if (ctx->scratch_n >= n) return MC_OK;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->scratch_bufs.release();
    ctx->scratch_n = 0;
    int rc = dalloc(ctx, ctx->scratch_bufs, &ctx->s_perm, n);
    if (!rc) rc = dalloc(ctx, ctx->scratch_bufs, &ctx->s_keys, n);
    if (!rc) rc = dalloc(ctx, ctx->scratch_bufs, &ctx->s_mat, n);
    if (!rc) rc = alloc_sort(ctx, ctx->scratch_bufs, ctx->s_sort, n);
    if (rc) {
        ctx->scratch_bufs.release();
        return rc;
    }
    ctx->scratch_n = n;
    return MC_OK;
}

static int timing_event_pair(mc_ctx *ctx, size_t k)
{
    while (ctx->ev_a.size() <= k) {
        hipEvent_t a, b;
        HIPCHK(hipEventCreate(&a));
        HIPCHK(hipEventCreate(&b));
        ctx->ev_a.push_back(a);
        ctx->ev_b.push_back(b);
    }
    return MC_OK;
}

int mc_run_batch(mc_ctx *ctx, uint64_t seed, uint64_t first_pid, uint64_t n, const mc_run_opts *opts_in)
{
    if (!ctx) return MC_EINVAL;
    if (!ctx->have_geom) return fail(ctx, MC_ESTATE, "mc_run_batch: materials and geometry first");
    if (n == 0) return fail(ctx, MC_EINVAL, "mc_run_batch: n must be >= 1");
    HIPCHK(hipSetDevice(ctx->device));
    mc_run_opts opts{};
    if (opts_in) opts = *opts_in;
    uint64_t cap64 = opts.in_flight ? opts.in_flight : kDefaultInFlight;
    cap64 = std::min(cap64, n);
    if (cap64 > (1ull << 30)) return fail(ctx, MC_EINVAL, "in_flight above 2^30");
    const uint64_t sort_min = opts.sort_min ? opts.sort_min : kDefaultSortMin;
    const int64_t max_events = opts.max_events > 0 ? opts.max_events : kDefaultMaxEvents;
    HistLog *log = static_cast<HistLog *>(opts.history_log);
    const uint32_t cap = (uint32_t)cap64;
    int rc = ensure_bank(ctx, cap);
    if (rc) return rc;
    hipStream_t st = ctx->stream;
    BankDev &b = ctx->bank;
    TallyDev tal = ctx->tal;
    tal.enabled = opts.no_tally ? 0 : 1;
    const GeomDev &g = ctx->geom;
    const bool mesh = g.tally_kind == TALLY_MESH;

    // reset per-batch state
    HIPCHK(launch_fill_u8(b.flags, cap, 0, st));
    const size_t row_bins = mesh ? 1 : (size_t)ctx->n_bins;
    HIPCHK(launch_fill_f64(tal.tl, (size_t)tal.rows * row_bins, 0.0, st));
    HIPCHK(launch_fill_f64(tal.coll, (size_t)tal.rows * row_bins, 0.0, st));
    HIPCHK(launch_fill_f64(tal.glob, (size_t)tal.rows * N_GLOBAL, 0.0, st));
    if (mesh) {
        HIPCHK(launch_fill_f64(tal.mesh_tl, (size_t)ctx->n_bins, 0.0, st));
        HIPCHK(launch_fill_f64(tal.mesh_coll, (size_t)ctx->n_bins, 0.0, st));
    }
    HIPCHK(launch_fill_u32(reinterpret_cast<uint32_t *>(ctx->ctr), 2 * sizeof(Counters) / 4, 0u, st));
    HIPCHK(launch_fill_u32(reinterpret_cast<uint32_t *>(ctx->dstat), 8, 0u, st));

    mc_stats s{};
    size_t n_timed = 0;
    HIPCHK(hipEventRecord(ctx->ev_batch0, st));
    uint64_t it = 0;
    // every history ends within max_events + 1 iterations of its start, so the
    // loop is bounded by the number of bank refills times that
    const uint64_t max_iter = (n / cap + 2) * ((uint64_t)max_events + 2);
    for (;; ++it) {
        if (it >= max_iter) return fail(ctx, MC_EHIP, "event loop did not terminate");
        const int cur = (int)(it & 1);
        HIPCHK(launch_slots_count(b, st));
        HIPCHK(launch_slots_queue(b, g, ctx->ctr, cur, first_pid, n, seed, st));
        HIPCHK(hipMemcpyAsync(ctx->ctr_host + cur, ctx->ctr + cur, sizeof(Counters), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        const Counters c = ctx->ctr_host[cur];
        if (c.nA == 0) {
            if (c.issued != n) return fail(ctx, MC_EHIP, "event loop ended before every history was issued");
            break;
        }
        Counters *dc = ctx->ctr + cur;
        const int64_t tail = tail_particles(ctx);
        if (tail > 0 && c.issued == n && (int64_t)c.nA <= tail) {
            // every history has started and few remain: finish them in one launch
            HIPCHK(launch_tail(b, ctx->xs, g, tal, dc, c.nA, seed, max_events, log, first_pid, ctx->dstat + 1, st));
            s.tail_particles = c.nA;
            ++it;
            break;
        }
        if (c.nL > 0) {
            LookupLaunch l;
            l.xs = ctx->xs;
            l.n_ptr = &dc->nL;
            l.n_bound = c.nL;
            l.E = b.E;
            l.mat = b.mat;
            l.Sa = b.Sa;
            l.Ss = b.Ss;
            l.flags = b.flags;
            l.nuc_count = ctx->dstat;
            l.ilp = lookup_ilp(ctx);
            const bool sort = (uint64_t)c.nL >= sort_min && sort_min != UINT64_MAX;
            if (sort) {
                HIPCHK(launch_sort(ctx->xs, b.L, &dc->nL, c.nL, b.E, b.mat, ctx->bank_sort, ctx->n_keys, b.Ls,
                                   b.Lkey, st));
                l.list = b.Ls;
                l.keys = b.Lkey;
                s.sorted_lookups += c.nL;
            } else {
                l.list = b.L;
            }
            if (opts.time_kernels) {
                rc = timing_event_pair(ctx, n_timed);
                if (rc) return rc;
                HIPCHK(hipEventRecord(ctx->ev_a[n_timed], st));
            }
            HIPCHK(launch_lookup(l, st));
            if (opts.time_kernels) {
                HIPCHK(hipEventRecord(ctx->ev_b[n_timed], st));
                ++n_timed;
            }
            s.lookups += c.nL;
            s.lookup_launches += 1;
        }
        HIPCHK(launch_advance(b, g, tal, dc, c.nA, seed, max_events, log ? 1 : 0, st));
        HIPCHK(launch_split(b, dc, c.nA, st));
        HIPCHK(launch_cross(b, g, tal, dc, c.nA, log, first_pid, ctx->dstat + 1, st));
        HIPCHK(launch_collide(b, ctx->xs, g, tal, dc, c.nA, seed, log, first_pid, st));
    }
    // batch statistics: per-workgroup rows summed in a fixed order
    const double inv_n = 1.0 / (double)n;
    if (mesh) {
        HIPCHK(launch_batch_stats(nullptr, 0, ctx->n_bins, tal.mesh_tl, ctx->partial, inv_n, ctx->S1[0],
                                  ctx->S2[0], st));
        HIPCHK(launch_batch_stats(nullptr, 0, ctx->n_bins, tal.mesh_coll, ctx->partial, inv_n, ctx->S1[1],
                                  ctx->S2[1], st));
    } else {
        HIPCHK(launch_batch_stats(tal.tl, tal.rows, ctx->n_bins, nullptr, ctx->partial, inv_n, ctx->S1[0],
                                  ctx->S2[0], st));
        HIPCHK(launch_batch_stats(tal.coll, tal.rows, ctx->n_bins, nullptr, ctx->partial, inv_n, ctx->S1[1],
                                  ctx->S2[1], st));
    }
    HIPCHK(launch_batch_stats(tal.glob, tal.rows, N_GLOBAL, nullptr, ctx->partial, inv_n, ctx->S1[2],
                              ctx->S2[2], st));
    HIPCHK(hipEventRecord(ctx->ev_batch1, st));
    unsigned long long dstat[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(dstat, ctx->dstat, sizeof(dstat), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, ctx->ev_batch0, ctx->ev_batch1));
    s.batch_ms = ms;
    for (size_t k = 0; k < n_timed; ++k) {
        float t = 0.f;
        HIPCHK(hipEventElapsedTime(&t, ctx->ev_a[k], ctx->ev_b[k]));
        s.lookup_ms += t;
    }
    s.iterations = it;
    s.nuclide_lookups = dstat[0];
    s.lost = dstat[1];
    s.lookup_bytes = 36ull * s.lookups + 56ull * s.nuclide_lookups;
    ctx->stats = s;
    ctx->n_batches += 1;
    ctx->histories += n;
    if (s.lost > opts.max_lost)
        return fail(ctx, MC_ELOST, std::to_string(s.lost) + " particles lost (event cap reached)");
    return MC_OK;
}

int mc_get_tallies(mc_ctx *ctx, int32_t tally_id, double *mean, double *stderr_, size_t n_bins,
                   mc_tally_meta *meta)
{
    if (!ctx) return MC_EINVAL;
    if (!ctx->have_geom) return fail(ctx, MC_ESTATE, "no geometry");
    if (tally_id < 0 || tally_id > 2) return fail(ctx, MC_EINVAL, "unknown tally id");
    const size_t nb = (tally_id == MC_T_GLOBAL) ? (size_t)N_GLOBAL : (size_t)ctx->n_bins;
    if (n_bins != nb) return fail(ctx, MC_EINVAL, "n_bins does not match the tally (" + std::to_string(nb) + ")");
    HIPCHK(hipSetDevice(ctx->device));
    std::vector<double> s1(nb), s2(nb);
    HIPCHK(hipMemcpyAsync(s1.data(), ctx->S1[tally_id], nb * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipMemcpyAsync(s2.data(), ctx->S2[tally_id], nb * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    const double B = (double)ctx->n_batches;
    for (size_t k = 0; k < nb; ++k) {
        const double m = B > 0 ? s1[k] / B : 0.0;
        if (mean) mean[k] = m;
        if (stderr_) stderr_[k] = (B > 1) ? std::sqrt(std::max(s2[k] / B - m * m, 0.0) / (B - 1.0)) : 0.0;
    }
    if (meta) {
        meta->n_batches = ctx->n_batches;
        meta->n_bins = nb;
        meta->histories = ctx->histories;
    }
    return MC_OK;
}

int mc_get_stats(mc_ctx *ctx, mc_stats *out)
{
    if (!ctx || !out) return MC_EINVAL;
    *out = ctx->stats;
    return MC_OK;
}

int mc_set_tuning(mc_ctx *ctx, const mc_tuning *t)
{
    if (!ctx || !t) return MC_EINVAL;
    if (t->lookup_ilp != 0 && t->lookup_ilp != 1 && t->lookup_ilp != 2 && t->lookup_ilp != 4)
        return fail(ctx, MC_EINVAL, "lookup_ilp must be 0, 1, 2 or 4");
    if (t->tail_particles < -1) return fail(ctx, MC_EINVAL, "tail_particles must be >= -1");
    ctx->tune = *t;
    return MC_OK;
}

int mc_get_tuning(mc_ctx *ctx, mc_tuning *t)
{
    if (!ctx || !t) return MC_EINVAL;
    *t = ctx->tune;
    t->lookup_ilp = lookup_ilp(ctx);
    t->tail_particles = (int32_t)tail_particles(ctx);
    return MC_OK;
}

int mc_set_timing(mc_ctx *ctx, int32_t on)
{
    if (!ctx) return MC_EINVAL;
    ctx->timing = on != 0;
    if (on) ctx->stats = mc_stats{};
    return MC_OK;
}

int mc_lookup_macro(mc_ctx *ctx, size_t n, const double *E, const int32_t *mat, double *sig_a, double *sig_s,
                    int32_t sorted)
{
    if (!ctx) return MC_EINVAL;
    if (!ctx->have_mat) return fail(ctx, MC_ESTATE, "mc_lookup_macro: no materials");
    if (n == 0) return MC_OK;
    if (n >= (1ull << 31) || !E || !mat) return fail(ctx, MC_EINVAL, "mc_lookup_macro: bad arguments");
    HIPCHK(hipSetDevice(ctx->device));
    LookupLaunch l;
    l.xs = ctx->xs;
    l.n_bound = (uint32_t)n;
    l.E = E;
    l.mat = mat;
    l.Sa = sig_a;
    l.Ss = sig_s;
    l.ilp = lookup_ilp(ctx);
    if (sorted) {
        int rc = ensure_scratch(ctx, n);
        if (rc) return rc;
        HIPCHK(launch_sort(ctx->xs, nullptr, nullptr, (uint32_t)n, E, mat, ctx->s_sort, ctx->n_keys, ctx->s_perm,
                           ctx->s_keys, ctx->stream));
        l.list = ctx->s_perm;
        l.keys = ctx->s_keys;
    }
    if (!ctx->timing) {
        HIPCHK(launch_lookup(l, ctx->stream));
        return MC_OK;
    }
    int rc = timing_event_pair(ctx, 0);
    if (rc) return rc;
    HIPCHK(launch_fill_u32(reinterpret_cast<uint32_t *>(ctx->dstat), 2, 0u, ctx->stream));
    l.nuc_count = ctx->dstat;
    HIPCHK(hipEventRecord(ctx->ev_a[0], ctx->stream));
    HIPCHK(launch_lookup(l, ctx->stream));
    HIPCHK(hipEventRecord(ctx->ev_b[0], ctx->stream));
    unsigned long long nuc = 0;
    HIPCHK(hipMemcpyAsync(&nuc, ctx->dstat, sizeof(nuc), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, ctx->ev_a[0], ctx->ev_b[0]));
    mc_stats &s = ctx->stats;
    s.lookups += n;
    s.nuclide_lookups += nuc;
    s.lookup_launches += 1;
    s.sorted_lookups += sorted ? n : 0;
    s.lookup_bytes += 36ull * n + 56ull * nuc;
    s.lookup_ms += ms;
    return MC_OK;
}

int mc_lookup_nuclides(mc_ctx *ctx, int32_t mat, size_t n, const double *E, int32_t *idx, double *sig_c,
                       double *sig_s)
{
    if (!ctx) return MC_EINVAL;
    if (!ctx->have_mat) return fail(ctx, MC_ESTATE, "mc_lookup_nuclides: no materials");
    if (mat < 0 || mat >= ctx->n_mat) return fail(ctx, MC_EINVAL, "mc_lookup_nuclides: material out of range");
    if (n == 0) return MC_OK;
    if (n >= (1ull << 31) || !E) return fail(ctx, MC_EINVAL, "mc_lookup_nuclides: bad arguments");
    HIPCHK(hipSetDevice(ctx->device));
    int rc = ensure_scratch(ctx, n);
    if (rc) return rc;
    HIPCHK(launch_fill_u32(reinterpret_cast<uint32_t *>(ctx->s_mat), n, (uint32_t)mat, ctx->stream));
    LookupLaunch l;
    l.xs = ctx->xs;
    l.n_bound = (uint32_t)n;
    l.E = E;
    l.mat = ctx->s_mat;
    l.idx_out = idx;
    l.sc_out = sig_c;
    l.ss_out = sig_s;
    l.ilp = lookup_ilp(ctx);
    HIPCHK(launch_lookup(l, ctx->stream));
    return MC_OK;
}

int mc_sort_queue(mc_ctx *ctx, size_t n, const double *E, const int32_t *mat, uint32_t *perm,
                  uint32_t *keys_sorted)
{
    if (!ctx) return MC_EINVAL;
    if (!ctx->have_mat) return fail(ctx, MC_ESTATE, "mc_sort_queue: no materials");
    if (n == 0) return MC_OK;
    if (n >= (1ull << 31) || !E || !mat || !perm) return fail(ctx, MC_EINVAL, "mc_sort_queue: bad arguments");
    HIPCHK(hipSetDevice(ctx->device));
    int rc = ensure_scratch(ctx, n);
    if (rc) return rc;
    HIPCHK(launch_sort(ctx->xs, nullptr, nullptr, (uint32_t)n, E, mat, ctx->s_sort, ctx->n_keys, perm,
                       keys_sorted ? keys_sorted : ctx->s_keys, ctx->stream));
    return MC_OK;
}

}  // extern "C"
