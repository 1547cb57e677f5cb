// mc_api.hip -- C ABI of libmc.so: context, data upload, the host side of the
// event loop and tally statistics.  Declarations and argument contracts are in
// include/mc.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <atomic>
#include <chrono>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/mc.h"
#include "mc_device.h"
#include "mc_internal.h"
#include "mc_physics.h"

using namespace mc;

namespace {

constexpr uint64_t kDefaultInFlight = 1ull << 22;         // analog bank: more particles, denser sorted queues
constexpr uint64_t kDefaultInFlightWindows = 1ull << 20;  // with weight windows (stacks of depth x slots)
constexpr uint64_t kMaxTunedInFlight = 1ull << 24;
constexpr uint64_t kDefaultSortMin = 262144;
constexpr uint64_t kSortNever = 1ull << 30;  // no queue is that long: never sort
constexpr int64_t kDefaultMaxEvents = 100000;
constexpr int64_t kDefaultTailParticles = 131072;

}  // namespace

// Scratch of the allocation-free lookup entry point (mc_lookup_macro_noalloc):
// a static device array, one copy per GPU, placed when the code object loads
// and held until the process ends.  In host code `scratch` names a host-side
// stand-in, not device memory: host code uses only the device address that
// hipGetSymbolAddress returns for it (taken once per device when a context is
// created on it, kept in noalloc_scratch_ptr).
static __device__ __align__(256) unsigned char scratch[MC_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void *g_noalloc_scratch[kMaxDevices] = {};

// The device address of `scratch` on the current device `device`, looked up
// on the first call for that device.
hipError_t noalloc_scratch_ptr(int device, void **out)
{
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_scratch[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_noalloc_scratch[device] = p;
    }
    *out = g_noalloc_scratch[device];
    return hipSuccess;
}
}  // namespace

// Device buffers of one part of a context, released together; they come from
// the context's allocator (mc_alloc) when it has one, else from hipMalloc.
struct Buffers {
    std::vector<void *> ptrs;
    const mc_ctx *owner = nullptr;  // set by the first dalloc
    void release();
};

struct mc_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    bool has_alloc = false;  // device memory from `alloc` (mc_create), else hipMalloc
    mc_alloc alloc{};

    // materials
    bool have_mat = false;
    Buffers mat_bufs;
    XsDev xs{};
    int32_t n_nuc = 0, n_mat = 0;
    std::vector<int32_t> mat_len;
    uint32_t n_keys = 0;  // n_mat * M sort keys
    std::vector<int32_t> nuc_glen;   // grid points per nuclide
    std::vector<uint32_t> nuc_goff;  // first point of each nuclide in the tables
    std::vector<int32_t> mat_nuc_host;  // nuclide ids of the materials, in order
    double emin = 0.0, emax = 0.0;   // energy range of the hash grid
    int32_t M = 0;                   // hash bins
    Buffers union_bufs;              // unionized grids (mc_set_union_grid)
    uint64_t union_bytes = 0;

    // windowed multipole data (mc_init_multipole)
    Buffers mp_bufs;
    MpDev mp{};
    bool have_mp = false;

    // reaction channels (tables, and the reaction-rate tally's batch sums)
    int32_t n_chan = 0;
    Buffers chan_bufs;

    // geometry and tallies
    bool have_geom = false;
    Buffers geom_bufs;
    GeomDev geom{};
    int32_t n_bins = 0;
    double *S1[4] = {nullptr, nullptr, nullptr, nullptr}, *S2[4] = {nullptr, nullptr, nullptr, nullptr};
    uint64_t n_batches = 0, histories = 0;
    double track_s1 = 0.0;  // host copy of S1 of the global track-length bin (mesh range check)

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
    void *noalloc_scratch = nullptr;  // this device's `scratch` (device address)

    std::vector<hipEvent_t> ev_a, ev_b;
    hipEvent_t ev_batch0 = nullptr, ev_batch1 = nullptr;
    hipEvent_t ev_ctr[2] = {nullptr, nullptr};  // an iteration's queue lengths are on the host

    // concurrent event loops (tuning field loops > 1): each a worker context
    // with its own stream, bank and counters, sharing this context's tables;
    // their tally rows are slices of one array so the batch sums them in order
    std::vector<mc_ctx *> workers;
    bool owns_stream = false;
    Buffers loop_bufs;
    TallyDev loop_tal{};         // [loops * rows] rows (mesh arrays shared)
    int32_t loop_n = 0, loop_rows = 0, loop_bins = -1, loop_chan_bins = -1;
    bool loop_mesh = false;
    double *loop_partial = nullptr;
    hipEvent_t ev_loop_start = nullptr;
    std::vector<hipEvent_t> ev_loop_done;
    Buffers batch_bufs;            // per-batch values of mc_run_batches
    double *batch_vals = nullptr;
    size_t batch_vals_n = 0;
    mc_stats stats{};
    bool timing = false;  // time the stand-alone lookups (mc_set_timing)
    mc_tuning tune{};      // launch shapes (0 = default)
    int n_cu = 256;        // compute units of the device
    std::string arch;      // gcnArchName of the device
    uint64_t xs_sig = 0, geom_sig = 0, set_sig = 0;  // signatures for the autotuner cache

    // problem set (batching layer)
    bool have_set = false;
    Buffers set_bufs, set_tile_bufs;
    XsDev set_xs{};
    SetDev set{};
    std::vector<SetProblem> set_probs;  // input order
    std::vector<int32_t> set_order;     // problems in tile order
    int32_t set_max_bins = 0;
    uint32_t set_tile_hist = 0;         // tile size the tiles were built for
    uint64_t set_batches = 0;
    uint64_t set_histories = 0;         // histories per batch over all problems
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    uint32_t graph_grid = 0, graph_tile = 0;
    int64_t graph_max_events = 0;

    // importance network
    bool have_mlp = false;
    Buffers mlp_bufs, mlp_scratch_bufs;
    float *theta = nullptr, *mom = nullptr, *vel = nullptr, *grad = nullptr, *inv_wsum = nullptr;
    uint16_t *W1b = nullptr, *W2b = nullptr, *W2tb = nullptr, *w3b = nullptr;
    int mlp_step = 0;
    float *mlp_partial = nullptr, *mlp_loss = nullptr;
    size_t mlp_scratch_n = 0;
    int32_t mlp_loss_cap = 0;

    // weight windows and the forward importance estimate
    mc_ww_desc ww_desc{};              // kind MC_WW_OFF, imp_nx 0: analog, no estimate
    Buffers ww_bufs, imp_bufs;
    WwDev ww{};                        // device arrays for ww_cap slots
    uint32_t ww_cap = 0;
    double *ln_src = nullptr;          // device scalar
    double *imp_num = nullptr, *imp_den = nullptr, *imp_cnt = nullptr;
    Buffers imp_sample_bufs;           // training samples built from the sums
    size_t imp_sample_cap = 0;
    float *imp_X = nullptr, *imp_T = nullptr, *imp_W = nullptr;
    int32_t *imp_n = nullptr;
    float *imp_range = nullptr;
};

void Buffers::release()
{
    for (void *p : ptrs) {
        if (owner && owner->has_alloc)
            owner->alloc.release(owner->alloc.user, p, owner->device, owner->stream);
        else
            (void)hipFree(p);
    }
    ptrs.clear();
}

static MlpDev mlp_dev(const mc_ctx *ctx)
{
    MlpDev m;
    m.theta = ctx->theta;
    m.W1 = ctx->W1b;
    m.W2 = ctx->W2b;
    m.W2t = ctx->W2tb;
    m.w3 = ctx->w3b;
    return m;
}

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
    b.owner = ctx;
    if (ctx->has_alloc) {
        q = ctx->alloc.alloc(ctx->alloc.user, count * sizeof(T), ctx->device, ctx->stream);
        if (!q) return fail(ctx, MC_ENOMEM, "allocator: " + std::to_string(count * sizeof(T)) + " bytes refused");
    } else {
        hipError_t e = hipMalloc(&q, count * sizeof(T));
        if (e != hipSuccess) return fail(ctx, MC_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
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

// FNV-1a over raw bytes: signatures of what the autotuner's timings depend on
static uint64_t fnv(uint64_t h, const void *p, size_t n)
{
    const unsigned char *c = static_cast<const unsigned char *>(p);
    for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
    return h;
}
template <class T>
static uint64_t fnv_vec(uint64_t h, const std::vector<T> &v)
{
    return fnv(h, v.data(), v.size() * sizeof(T));
}
static uint64_t geom_signature(uint64_t h, const GeomDev &g)
{
    const int32_t ints[] = {g.kind, g.nx, g.ny, g.n_layers, g.src_kind, g.tally_kind, g.n_bins};
    const double dbl[] = {g.pitch, g.radius, g.z0, g.z1, g.src_E, g.e_cut};
    return fnv(fnv(h, ints, sizeof(ints)), dbl, sizeof(dbl));
}

extern "C" {

const char *mc_version(void) { return "mc355 0.1 (gfx950)"; }

int mc_create(mc_ctx **out, int device, void *hip_stream, const mc_alloc *alloc)
{
    if (!out) return MC_EINVAL;
    *out = nullptr;
    if (alloc && (!alloc->alloc || !alloc->release)) return MC_EINVAL;
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
    if (alloc) {
        ctx->has_alloc = true;
        ctx->alloc = *alloc;
    }
    ctx->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    ctx->arch = prop.gcnArchName;
    int rc = noalloc_scratch_ptr(device, &ctx->noalloc_scratch) == hipSuccess ? MC_OK : MC_EHIP;
    if (!rc) rc = dalloc(ctx, ctx->misc_bufs, &ctx->ctr, 2);
    if (!rc) rc = dalloc(ctx, ctx->misc_bufs, &ctx->dstat, 4);
    if (!rc && hipHostMalloc((void **)&ctx->ctr_host, 2 * sizeof(Counters), hipHostMallocDefault) != hipSuccess)
        rc = MC_ENOMEM;
    if (!rc && (hipEventCreate(&ctx->ev_batch0) != hipSuccess || hipEventCreate(&ctx->ev_batch1) != hipSuccess))
        rc = MC_EHIP;
    for (int k = 0; k < 2 && !rc; ++k)
        if (hipEventCreateWithFlags(&ctx->ev_ctr[k], hipEventDisableTiming) != hipSuccess) rc = MC_EHIP;
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
    for (mc_ctx *w : ctx->workers) mc_destroy(w);
    ctx->workers.clear();
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    ctx->loop_bufs.release();
    ctx->batch_bufs.release();
    ctx->union_bufs.release();
    ctx->mp_bufs.release();
    if (ctx->ev_loop_start) (void)hipEventDestroy(ctx->ev_loop_start);
    for (hipEvent_t e : ctx->ev_loop_done) (void)hipEventDestroy(e);
    ctx->mat_bufs.release();
    ctx->geom_bufs.release();
    ctx->bank_bufs.release();
    ctx->misc_bufs.release();
    ctx->scratch_bufs.release();
    ctx->set_bufs.release();
    ctx->set_tile_bufs.release();
    ctx->mlp_bufs.release();
    ctx->mlp_scratch_bufs.release();
    ctx->ww_bufs.release();
    ctx->imp_bufs.release();
    ctx->imp_sample_bufs.release();
    if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    if (ctx->ctr_host) (void)hipHostFree(ctx->ctr_host);
    for (hipEvent_t e : ctx->ev_a) (void)hipEventDestroy(e);
    for (hipEvent_t e : ctx->ev_b) (void)hipEventDestroy(e);
    if (ctx->ev_batch0) (void)hipEventDestroy(ctx->ev_batch0);
    if (ctx->ev_batch1) (void)hipEventDestroy(ctx->ev_batch1);
    for (hipEvent_t e : ctx->ev_ctr)
        if (e) (void)hipEventDestroy(e);
    if (ctx->owns_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
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

// ---------------------------------------------------------------------------
// cross-section tables: validation and host layout, shared by the single
// problem and the problem set
// ---------------------------------------------------------------------------
struct NuclideInput {
    int32_t n_nuc;
    const int32_t *grid_len;
    const double *const *E, *const *sig_c, *const *sig_s;
    const double *awr;
    int32_t n_mat;
    const int32_t *mat_len, *mat_nuc;
    const double *mat_dens;
};

struct HostXs {
    std::vector<double> Eg, xs, awr;
    std::vector<int32_t> moff{0}, mnucid, mat_len;
    std::vector<MatNuc> mnuc;
    std::vector<uint64_t> hoff;
    std::vector<uint32_t> hash;
    std::vector<const double *> grids;   // per nuclide (host, for the bounds)
    std::vector<int32_t> glen;
    std::vector<uint32_t> goff;
    double emin = INFINITY, emax = 0.0;
};

// Validate one problem's nuclides and materials and append them (nuclide and
// material ids shifted by what is already there).
static int append_xs(mc_ctx *ctx, HostXs &H, const NuclideInput &in, const std::string &who)
{
    if (in.n_nuc < 1 || !in.grid_len || !in.E || !in.sig_c || !in.sig_s || !in.awr || in.n_mat < 1 ||
        !in.mat_len || !in.mat_nuc || !in.mat_dens)
        return fail(ctx, MC_EINVAL, who + "missing array or non-positive count");
    const int32_t nuc_base = (int32_t)H.glen.size();
    for (int32_t k = 0; k < in.n_nuc; ++k) {
        const int32_t n = in.grid_len[k];
        const std::string nk = who + "nuclide " + std::to_string(k) + ": ";
        if (n < 2 || !in.E[k] || !in.sig_c[k] || !in.sig_s[k]) return fail(ctx, MC_EINVAL, nk + "grid shorter than 2 points");
        if (!(in.awr[k] > 0.0) || !std::isfinite(in.awr[k])) return fail(ctx, MC_EINVAL, nk + "mass ratio must be > 0");
        for (int32_t j = 0; j < n; ++j) {
            if (!std::isfinite(in.E[k][j]) || !(in.E[k][j] > 0.0))
                return fail(ctx, MC_EINVAL, nk + "energy not finite and > 0");
            if (j && !(in.E[k][j] > in.E[k][j - 1]))
                return fail(ctx, MC_EINVAL, nk + "grid not strictly increasing at point " + std::to_string(j));
            if (!(in.sig_c[k][j] >= 0.0) || !(in.sig_s[k][j] >= 0.0) || !std::isfinite(in.sig_c[k][j]) ||
                !std::isfinite(in.sig_s[k][j]))
                return fail(ctx, MC_EINVAL, nk + "cross section < 0 or not finite");
        }
        if ((uint64_t)H.Eg.size() + (uint64_t)n >= (1ull << 32))
            return fail(ctx, MC_EINVAL, "more than 2^32 grid points in total");
        H.goff.push_back((uint32_t)H.Eg.size());
        H.glen.push_back(n);
        H.grids.push_back(in.E[k]);
        for (int32_t j = 0; j < n; ++j) {
            H.Eg.push_back(in.E[k][j]);
            H.xs.push_back(in.sig_c[k][j]);
            H.xs.push_back(in.sig_s[k][j]);
        }
        H.awr.push_back(in.awr[k]);
        H.emin = std::min(H.emin, in.E[k][0]);
        H.emax = std::max(H.emax, in.E[k][n - 1]);
    }
    uint64_t q = 0;
    for (int32_t m = 0; m < in.n_mat; ++m) {
        const std::string mk = who + "material " + std::to_string(m) + ": ";
        if (in.mat_len[m] < 1) return fail(ctx, MC_EINVAL, mk + "no nuclides");
        for (int32_t j = 0; j < in.mat_len[m]; ++j, ++q) {
            const int32_t k = in.mat_nuc[q];
            const double d = in.mat_dens[q];
            if (k < 0 || k >= in.n_nuc) return fail(ctx, MC_EINVAL, mk + "unknown nuclide id " + std::to_string(k));
            if (!(d > 0.0) || !std::isfinite(d)) return fail(ctx, MC_EINVAL, mk + "density must be > 0");
            H.mnucid.push_back(nuc_base + k);
            H.mnuc.push_back(MatNuc{0u, 0u, d});  // grid placement filled in finish_xs
        }
        H.mat_len.push_back(in.mat_len[m]);
        H.moff.push_back(H.moff.back() + in.mat_len[m]);
    }
    return MC_OK;
}

// Hash bounds of every material over the common [emin, emax] with M bins.
static int finish_xs(mc_ctx *ctx, HostXs &H, int32_t M)
{
    const size_t n_mat = H.mat_len.size();
    if ((uint64_t)n_mat * (uint64_t)M >= (1ull << 32)) return fail(ctx, MC_EINVAL, "n_mat * n_hash_bins must stay below 2^32");
    const size_t n_nuc = H.glen.size();
    std::vector<int32_t> lo(n_nuc * (size_t)(M + 1));
    for (size_t k = 0; k < n_nuc; ++k) build_bounds(H.grids[k], H.glen[k], H.emin, H.emax, M, &lo[k * (M + 1)]);
    uint64_t pairs = 0;  // brackets (lo_b, lo_b+1) per material, bin and nuclide
    H.hoff.resize(n_mat);
    for (size_t m = 0; m < n_mat; ++m) {
        H.hoff[m] = pairs;
        pairs += (uint64_t)M * (uint64_t)H.mat_len[m];
    }
    H.hash.assign(2 * pairs, 0u);
    for (size_t m = 0; m < n_mat; ++m) {
        const int32_t nk = H.mat_len[m];
        for (int32_t q = 0; q < nk; ++q) {
            const int32_t k = H.mnucid[H.moff[m] + q];
            MatNuc &mn = H.mnuc[H.moff[m] + q];
            mn.off = H.goff[k];
            mn.len = (uint32_t)H.glen[k];
            for (int32_t b = 0; b < M; ++b) {
                const uint64_t at = 2 * (H.hoff[m] + (uint64_t)b * nk + q);
                H.hash[at] = (uint32_t)lo[(size_t)k * (M + 1) + b];
                H.hash[at + 1] = (uint32_t)lo[(size_t)k * (M + 1) + b + 1];
            }
        }
    }
    return MC_OK;
}

static int upload_xs(mc_ctx *ctx, const HostXs &H, int32_t M, Buffers &B, XsDev &x)
{
    double *d_Eg, *d_awr;
    double2 *d_xs;
    int32_t *d_moff, *d_mnucid;
    MatNuc *d_mnuc;
    uint2 *d_hash;
    uint64_t *d_hoff;
    int rc = upload(ctx, B, &d_Eg, H.Eg.data(), H.Eg.size());
    if (!rc) rc = upload(ctx, B, &d_xs, reinterpret_cast<const double2 *>(H.xs.data()), H.Eg.size());
    if (!rc) rc = upload(ctx, B, &d_awr, H.awr.data(), H.awr.size());
    if (!rc) rc = upload(ctx, B, &d_moff, H.moff.data(), H.moff.size());
    if (!rc) rc = upload(ctx, B, &d_mnucid, H.mnucid.data(), H.mnucid.size());
    if (!rc) rc = upload(ctx, B, &d_mnuc, H.mnuc.data(), H.mnuc.size());
    if (!rc) rc = upload(ctx, B, &d_hash, reinterpret_cast<const uint2 *>(H.hash.data()), H.hash.size() / 2);
    if (!rc) rc = upload(ctx, B, &d_hoff, H.hoff.data(), H.hoff.size());
    if (rc) return rc;
    x = XsDev{};
    x.Eg = d_Eg;
    x.xs = d_xs;
    x.awr = d_awr;
    x.mat_off = d_moff;
    x.mat_nuc = d_mnucid;
    x.mnuc = d_mnuc;
    x.hash = d_hash;
    x.hash_off = d_hoff;
    x.n_mat = (int32_t)H.mat_len.size();
    x.M = M;
    x.ln_emin = std::log(H.emin);
    x.inv_delta = (double)M / std::log(H.emax / H.emin);
    x.div_safe = H.emin >= 0x1p-100 && H.emax <= 0x1p100 ? 1 : 0;
    return MC_OK;
}

int mc_init_materials(mc_ctx *ctx, int32_t n_nuc, const int32_t *grid_len, const double *const *E,
                      const double *const *sig_c, const double *const *sig_s, const double *awr,
                      int32_t n_mat, const int32_t *mat_len, const int32_t *mat_nuc, const double *mat_dens,
                      int32_t n_hash_bins)
{
    if (!ctx) return MC_EINVAL;
    if (n_hash_bins < 1) return fail(ctx, MC_EINVAL, "mc_init_materials: n_hash_bins must be >= 1");
    HIPCHK(hipSetDevice(ctx->device));
    HostXs H;
    const NuclideInput in{n_nuc, grid_len, E, sig_c, sig_s, awr, n_mat, mat_len, mat_nuc, mat_dens};
    int rc = append_xs(ctx, H, in, "mc_init_materials: ");
    if (!rc) rc = finish_xs(ctx, H, n_hash_bins);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->mat_bufs.release();
    ctx->chan_bufs.release();  // new tables: no reaction channels until mc_init_channels
    ctx->union_bufs.release();  // ... and no unionized grids until mc_set_union_grid
    ctx->union_bytes = 0;
    ctx->n_chan = 0;
    ctx->S1[3] = ctx->S2[3] = nullptr;
    ctx->have_mat = false;
    ctx->have_geom = false;
    rc = upload_xs(ctx, H, n_hash_bins, ctx->mat_bufs, ctx->xs);
    ctx->xs.n_chan = 0;
    ctx->xs.xc = nullptr;
    if (rc) {
        ctx->mat_bufs.release();
        return rc;
    }
    ctx->n_keys = (uint32_t)((uint64_t)n_mat * (uint64_t)n_hash_bins);
    ctx->xs_sig = fnv(fnv_vec(fnv_vec(fnv_vec(1469598103934665603ull, H.glen), H.mnucid), H.awr), &n_hash_bins,
                      sizeof(n_hash_bins));
    ctx->n_nuc = n_nuc;
    ctx->n_mat = n_mat;
    ctx->mat_len.assign(mat_len, mat_len + n_mat);
    ctx->nuc_glen = H.glen;
    ctx->nuc_goff = H.goff;
    ctx->mat_nuc_host = H.mnucid;
    ctx->emin = H.emin;
    ctx->emax = H.emax;
    ctx->M = n_hash_bins;
    ctx->have_mat = true;
    return MC_OK;
}

// Adds the counters of q (one batch or one loop) into a; the wall time, the
// iteration count and the algorithmic lookup bytes are set by the caller.
static void add_stats(mc_stats &a, const mc_stats &q)
{
    a.lookups += q.lookups;
    a.nuclide_lookups += q.nuclide_lookups;
    a.lookup_launches += q.lookup_launches;
    a.sorted_lookups += q.sorted_lookups;
    a.lost += q.lost;
    a.lookup_ms += q.lookup_ms;
    a.tail_particles += q.tail_particles;
    a.mesh_underflow += q.mesh_underflow;
    a.flights += q.flights;
    a.advance_ms += q.advance_ms;
    a.cross_ms += q.cross_ms;
    a.collide_ms += q.collide_ms;
}

static int timing_event_pair(mc_ctx *ctx, size_t k);

// Coefficients a_1 .. a_N of the rational Faddeeva series (Weideman 1994):
// the cosine coefficients of f(t) = exp(-t^2) (L^2 + t^2) on t = L tan(theta/2),
// by a plain sum over theta_k = k pi / M, k = -M+1 .. M-1, M = 2N,
// L = sqrt(N / sqrt 2).
static void faddeeva_coefficients(double *a, double &L)
{
    const int N = FAD_N, M = 2 * N;
    L = std::sqrt(std::sqrt((double)N * (double)N / 2.0));
    const double pi = 3.14159265358979323846;
    for (int n = 1; n <= N; ++n) {
        double s = 0.0;
        for (int k = -M + 1; k <= M - 1; ++k) {
            const double t = L * std::tan((double)k * pi / (double)M / 2.0);
            s += std::exp(-t * t) * (L * L + t * t) * std::cos(pi * (double)n * (double)k / (double)M);
        }
        a[n - 1] = s / (2.0 * (double)M);
    }
}

int mc_init_multipole(mc_ctx *ctx, int32_t n_nuc, const mc_mp_nuclide *nucs, const double *awr, int32_t n_mat,
                      const int32_t *mat_len, const int32_t *mat_nuc, const double *mat_dens, const double *mat_temp)
{
    if (!ctx) return MC_EINVAL;
    if (n_nuc < 1 || !nucs || !awr || n_mat < 1 || !mat_len || !mat_nuc || !mat_dens || !mat_temp)
        return fail(ctx, MC_EINVAL, "mc_init_multipole: missing array or non-positive count");
    std::vector<MpNuc> nd(n_nuc);
    std::vector<double> poles, rc, rs, bgc, bgs;
    std::vector<int32_t> win;
    for (int32_t k = 0; k < n_nuc; ++k) {
        const mc_mp_nuclide &x = nucs[k];
        const std::string who = "mc_init_multipole: nuclide " + std::to_string(k) + ": ";
        if (x.n_poles < 0 || x.n_windows < 1 || x.n_bg < 0 || x.n_bg > 8) return fail(ctx, MC_EINVAL, who + "counts");
        if (!(x.u_lo > 0.0) || !(x.u_hi > x.u_lo)) return fail(ctx, MC_EINVAL, who + "window range");
        if (!(awr[k] > 0.0)) return fail(ctx, MC_EINVAL, who + "awr must be > 0");
        if (!x.win || (x.n_poles > 0 && (!x.poles || !x.res_c || !x.res_s)) || (x.n_bg > 0 && (!x.bg_c || !x.bg_s)))
            return fail(ctx, MC_EINVAL, who + "missing array");
        for (int32_t w = 0; w < x.n_windows; ++w)
            if (x.win[2 * w] < 0 || x.win[2 * w] > x.win[2 * w + 1] || x.win[2 * w + 1] > x.n_poles)
                return fail(ctx, MC_EINVAL, who + "window " + std::to_string(w) + " pole range");
        for (int32_t j = 0; j < 2 * x.n_poles; ++j)
            if (!std::isfinite(x.poles[j]) || !std::isfinite(x.res_c[j]) || !std::isfinite(x.res_s[j]))
                return fail(ctx, MC_EINVAL, who + "non-finite pole data");
        for (int32_t j = 0; j < x.n_poles; ++j)
            if (!(x.poles[2 * j + 1] < 0.0)) return fail(ctx, MC_EINVAL, who + "poles need Im p < 0");
        nd[k].p_off = (uint32_t)(poles.size() / 2);
        nd[k].w_off = (uint32_t)(win.size() / 2);
        nd[k].bg_off = (uint32_t)bgc.size();
        nd[k].n_windows = x.n_windows;
        nd[k].n_bg = x.n_bg;
        nd[k].u_lo = x.u_lo;
        nd[k].du = (x.u_hi - x.u_lo) / (double)x.n_windows;
        poles.insert(poles.end(), x.poles, x.poles + 2 * x.n_poles);
        rc.insert(rc.end(), x.res_c, x.res_c + 2 * x.n_poles);
        rs.insert(rs.end(), x.res_s, x.res_s + 2 * x.n_poles);
        win.insert(win.end(), x.win, x.win + 2 * x.n_windows);
        bgc.insert(bgc.end(), x.bg_c, x.bg_c + (size_t)x.n_windows * x.n_bg);
        bgs.insert(bgs.end(), x.bg_s, x.bg_s + (size_t)x.n_windows * x.n_bg);
    }
    std::vector<int32_t> moff{0};
    std::vector<double> beta;
    constexpr double kB = 8.617333262e-5;  // eV / K
    for (int32_t m = 0; m < n_mat; ++m) {
        if (mat_len[m] < 1) return fail(ctx, MC_EINVAL, "mc_init_multipole: empty material");
        if (!(mat_temp[m] > 0.0)) return fail(ctx, MC_EINVAL, "mc_init_multipole: temperatures must be > 0 K");
        for (int32_t q = 0; q < mat_len[m]; ++q) {
            const int32_t i = moff.back() + q, k = mat_nuc[i];
            if (k < 0 || k >= n_nuc) return fail(ctx, MC_EINVAL, "mc_init_multipole: unknown nuclide id");
            if (!(mat_dens[i] > 0.0)) return fail(ctx, MC_EINVAL, "mc_init_multipole: densities must be > 0");
            beta.push_back(std::sqrt(awr[k] / (kB * mat_temp[m])));
        }
        moff.push_back(moff.back() + mat_len[m]);
    }
    double fa[FAD_N], fL = 0.0;
    faddeeva_coefficients(fa, fL);
    HIPCHK(hipSetDevice(ctx->device));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->mp_bufs.release();
    ctx->have_mp = false;
    Buffers &B = ctx->mp_bufs;
    MpDev d{};
    MpNuc *d_nd = nullptr;
    double2 *d_p = nullptr, *d_rc = nullptr, *d_rs = nullptr;
    int2 *d_w = nullptr;
    double *d_bgc = nullptr, *d_bgs = nullptr, *d_dens = nullptr, *d_beta = nullptr, *d_fa = nullptr;
    int32_t *d_moff = nullptr, *d_mnuc = nullptr;
    const size_t np = std::max<size_t>(poles.size() / 2, 1);
    poles.resize(2 * np, -1.0);
    rc.resize(2 * np, 0.0);
    rs.resize(2 * np, 0.0);
    if (bgc.empty()) {
        bgc.push_back(0.0);
        bgs.push_back(0.0);
    }
    int rc_ = upload(ctx, B, &d_nd, nd.data(), nd.size());
    if (!rc_) rc_ = upload(ctx, B, &d_p, reinterpret_cast<const double2 *>(poles.data()), np);
    if (!rc_) rc_ = upload(ctx, B, &d_rc, reinterpret_cast<const double2 *>(rc.data()), np);
    if (!rc_) rc_ = upload(ctx, B, &d_rs, reinterpret_cast<const double2 *>(rs.data()), np);
    if (!rc_) rc_ = upload(ctx, B, &d_w, reinterpret_cast<const int2 *>(win.data()), win.size() / 2);
    if (!rc_) rc_ = upload(ctx, B, &d_bgc, bgc.data(), bgc.size());
    if (!rc_) rc_ = upload(ctx, B, &d_bgs, bgs.data(), bgs.size());
    if (!rc_) rc_ = upload(ctx, B, &d_moff, moff.data(), moff.size());
    if (!rc_) rc_ = upload(ctx, B, &d_mnuc, mat_nuc, (size_t)moff.back());
    if (!rc_) rc_ = upload(ctx, B, &d_dens, mat_dens, (size_t)moff.back());
    if (!rc_) rc_ = upload(ctx, B, &d_beta, beta.data(), beta.size());
    if (!rc_) rc_ = upload(ctx, B, &d_fa, fa, (size_t)FAD_N);
    if (rc_) {
        B.release();
        return rc_;
    }
    d.nuc = d_nd;
    d.poles = d_p;
    d.rc = d_rc;
    d.rs = d_rs;
    d.win = d_w;
    d.bgc = d_bgc;
    d.bgs = d_bgs;
    d.mat_off = d_moff;
    d.mat_nuc = d_mnuc;
    d.mat_dens = d_dens;
    d.mat_beta = d_beta;
    d.fa = d_fa;
    d.fL = fL;
    d.n_mat = n_mat;
    ctx->mp = d;
    ctx->have_mp = true;
    return MC_OK;
}

int mc_lookup_multipole(mc_ctx *ctx, size_t n, const double *E, const int32_t *mat, double *sig_a, double *sig_s,
                        uint64_t *poles_evaluated)
{
    if (!ctx) return MC_EINVAL;
    if (!ctx->have_mp) return fail(ctx, MC_ESTATE, "mc_lookup_multipole: no multipole data");
    if (n == 0) return MC_OK;
    if (n >= (1ull << 31) || !E || !mat || !sig_a || !sig_s)
        return fail(ctx, MC_EINVAL, "mc_lookup_multipole: bad arguments");
    HIPCHK(hipSetDevice(ctx->device));
    unsigned long long *cnt = poles_evaluated ? ctx->dstat + 2 : nullptr;
    if (cnt) HIPCHK(launch_fill_u32(reinterpret_cast<uint32_t *>(cnt), 2, 0u, ctx->stream));
    if (ctx->timing) {
        int rc = timing_event_pair(ctx, 0);
        if (rc) return rc;
        HIPCHK(hipEventRecord(ctx->ev_a[0], ctx->stream));
    }
    HIPCHK(launch_lookup_mp(ctx->mp, (uint32_t)n, E, mat, sig_a, sig_s, cnt, ctx->stream));
    if (ctx->timing) {
        HIPCHK(hipEventRecord(ctx->ev_b[0], ctx->stream));
        HIPCHK(hipEventSynchronize(ctx->ev_b[0]));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, ctx->ev_a[0], ctx->ev_b[0]));
        ctx->stats.lookups += n;
        ctx->stats.lookup_launches += 1;
        ctx->stats.lookup_ms += ms;
    }
    if (cnt) {
        unsigned long long c = 0;
        HIPCHK(hipMemcpyAsync(&c, cnt, sizeof(c), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        *poles_evaluated = c;
    }
    return MC_OK;
}

int mc_set_union_grid(mc_ctx *ctx, int32_t on, uint64_t *bytes)
{
    if (!ctx) return MC_EINVAL;
    if (!ctx->have_mat) return fail(ctx, MC_ESTATE, "mc_set_union_grid: materials first");
    HIPCHK(hipSetDevice(ctx->device));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->union_bufs.release();
    ctx->union_bytes = 0;
    ctx->xs.um = nullptr;
    ctx->xs.ug = nullptr;
    ctx->xs.uh = nullptr;
    ctx->xs.ui = nullptr;
    if (bytes) *bytes = 0;
    if (!on) return MC_OK;
    // the nuclide grids, back from the device
    const size_t pts = ctx->nuc_goff.back() + (size_t)ctx->nuc_glen.back();
    std::vector<double> Eg(pts);
    HIPCHK(hipMemcpy(Eg.data(), ctx->xs.Eg, pts * sizeof(double), hipMemcpyDeviceToHost));
    const int32_t M = ctx->M;
    const double delta = std::log(ctx->emax / ctx->emin) / (double)M;
    std::vector<UnionMat> um(ctx->n_mat);
    std::vector<double> ug;
    std::vector<uint32_t> uh, ui;
    size_t q_base = 0;
    for (int32_t m = 0; m < ctx->n_mat; ++m) {
        const int32_t nk = ctx->mat_len[m];
        std::vector<double> U;
        for (int32_t q = 0; q < nk; ++q) {
            const int32_t k = ctx->mat_nuc_host[q_base + q];
            const double *g = Eg.data() + ctx->nuc_goff[k];
            U.insert(U.end(), g, g + ctx->nuc_glen[k]);
        }
        std::sort(U.begin(), U.end());
        U.erase(std::unique(U.begin(), U.end()), U.end());
        const size_t NU = U.size();
        if (NU * (size_t)nk > (size_t)1 << 34 || NU >= (1ull << 32))
            return fail(ctx, MC_EINVAL, "mc_set_union_grid: union grid of material " + std::to_string(m) + " too large");
        um[m].g_off = ug.size();
        um[m].i_off = ui.size();
        um[m].n = (uint32_t)NU;
        um[m].h_off = (uint32_t)uh.size();
        for (int32_t b = 0; b < M; ++b)
            uh.push_back((uint32_t)host_grid_index(U.data(), (int32_t)NU, ctx->emin * std::exp((double)b * delta)));
        uh.push_back((uint32_t)(NU - 2));
        // rows: i_q(U_u) = max{j : E_j <= U_u} clamped to [0, N - 2], one walk per nuclide
        const size_t base = ui.size();
        ui.resize(base + NU * (size_t)nk);
        for (int32_t q = 0; q < nk; ++q) {
            const int32_t k = ctx->mat_nuc_host[q_base + q];
            const double *g = Eg.data() + ctx->nuc_goff[k];
            const int32_t N = ctx->nuc_glen[k];
            int32_t j = 0;
            for (size_t u = 0; u < NU; ++u) {
                while (j + 1 < N && g[j + 1] <= U[u]) ++j;
                ui[base + u * (size_t)nk + q] = (uint32_t)std::min(j, N - 2);
            }
        }
        ug.insert(ug.end(), U.begin(), U.end());
        q_base += (size_t)nk;
    }
    UnionMat *d_um = nullptr;
    double *d_ug = nullptr;
    uint32_t *d_uh = nullptr, *d_ui = nullptr;
    Buffers &B = ctx->union_bufs;
    int rc = upload(ctx, B, &d_um, um.data(), um.size());
    if (!rc) rc = upload(ctx, B, &d_ug, ug.data(), ug.size());
    if (!rc) rc = upload(ctx, B, &d_uh, uh.data(), uh.size());
    if (!rc) rc = upload(ctx, B, &d_ui, ui.data(), ui.size());
    if (rc) {
        B.release();
        return rc;
    }
    ctx->xs.um = d_um;
    ctx->xs.ug = d_ug;
    ctx->xs.uh = d_uh;
    ctx->xs.ui = d_ui;
    ctx->union_bytes = ug.size() * sizeof(double) + (uh.size() + ui.size()) * sizeof(uint32_t);
    if (bytes) *bytes = ctx->union_bytes;
    return MC_OK;
}

int mc_init_channels(mc_ctx *ctx, int32_t n_chan, const double *const *sig_x)
{
    if (!ctx) return MC_EINVAL;
    if (!ctx->have_mat) return fail(ctx, MC_ESTATE, "mc_init_channels: materials first");
    if (n_chan < 0 || n_chan > MAX_CHAN)
        return fail(ctx, MC_EINVAL, "mc_init_channels: n_chan must be in [0, " + std::to_string(MAX_CHAN) + "]");
    if (n_chan > 0 && !sig_x) return fail(ctx, MC_EINVAL, "mc_init_channels: missing sig_x");
    std::vector<double> xc;
    if (n_chan > 0) {
        const size_t pts = ctx->nuc_goff.back() + (size_t)ctx->nuc_glen.back();
        xc.resize(pts * (size_t)n_chan);
        for (int32_t k = 0; k < ctx->n_nuc; ++k) {
            if (!sig_x[k]) return fail(ctx, MC_EINVAL, "mc_init_channels: missing nuclide " + std::to_string(k));
            const size_t cnt = (size_t)ctx->nuc_glen[k] * (size_t)n_chan;
            for (size_t j = 0; j < cnt; ++j) {
                const double v = sig_x[k][j];
                if (!(v >= 0.0) || !std::isfinite(v))
                    return fail(ctx, MC_EINVAL, "mc_init_channels: negative or non-finite value, nuclide " +
                                                    std::to_string(k));
            }
            std::memcpy(xc.data() + (size_t)ctx->nuc_goff[k] * (size_t)n_chan, sig_x[k], cnt * sizeof(double));
        }
    }
    HIPCHK(hipSetDevice(ctx->device));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->chan_bufs.release();
    ctx->n_chan = 0;
    ctx->xs.n_chan = 0;
    ctx->xs.xc = nullptr;
    ctx->S1[3] = ctx->S2[3] = nullptr;
    if (n_chan == 0) return MC_OK;
    double *d = nullptr;
    const size_t nb = (size_t)ctx->n_mat * (size_t)n_chan;
    int rc = upload(ctx, ctx->chan_bufs, &d, xc.data(), xc.size());
    if (!rc) rc = dalloc(ctx, ctx->chan_bufs, &ctx->S1[3], nb);
    if (!rc) rc = dalloc(ctx, ctx->chan_bufs, &ctx->S2[3], nb);
    if (rc) {
        ctx->chan_bufs.release();
        ctx->S1[3] = ctx->S2[3] = nullptr;
        return rc;
    }
    ctx->xs.n_chan = n_chan;
    ctx->xs.xc = d;
    ctx->n_chan = n_chan;
    HIPCHK(launch_fill_f64(ctx->S1[3], nb, 0.0, ctx->stream));
    HIPCHK(launch_fill_f64(ctx->S2[3], nb, 0.0, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return MC_OK;
}

static int reset_tallies(mc_ctx *ctx)
{
    for (int t = 0; t < 4; ++t) {
        if (t == 3 && !ctx->n_chan) break;
        const size_t n = (t == 2) ? (size_t)N_GLOBAL
                                  : (t == 3 ? (size_t)ctx->n_mat * (size_t)ctx->n_chan : (size_t)ctx->n_bins);
        HIPCHK(launch_fill_f64(ctx->S1[t], n, 0.0, ctx->stream));
        HIPCHK(launch_fill_f64(ctx->S2[t], n, 0.0, ctx->stream));
    }
    if (ctx->imp_num) {
        const size_t cells = (size_t)ctx->ww_desc.imp_nx * (size_t)ctx->ww_desc.imp_ne;
        HIPCHK(launch_fill_f64(ctx->imp_num, cells, 0.0, ctx->stream));
        HIPCHK(launch_fill_f64(ctx->imp_den, cells, 0.0, ctx->stream));
        HIPCHK(launch_fill_f64(ctx->imp_cnt, cells, 0.0, ctx->stream));
    }
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->n_batches = 0;
    ctx->histories = 0;
    ctx->track_s1 = 0.0;
    return MC_OK;
}

int mc_reset_tallies(mc_ctx *ctx)
{
    if (!ctx) return MC_EINVAL;
    if (!ctx->have_geom) return fail(ctx, MC_ESTATE, "no geometry");
    HIPCHK(hipSetDevice(ctx->device));
    return reset_tallies(ctx);
}

// Validate a geometry description whose material ids lie in [0, n_mat), and
// fill g (material ids shifted by mat_base; arrays uploaded into B).
static int build_geometry(mc_ctx *ctx, const mc_geometry_desc *d, int32_t n_mat, int32_t mat_base, Buffers &B,
                          GeomDev &g, const std::string &who)
{
    auto bad = [&](const std::string &m) { return fail(ctx, MC_EINVAL, who + m); };
    auto mat_ok = [&](int32_t m) { return m >= 0 && m < n_mat; };
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
    if (d->tally_kind != MC_TALLY_MESH && n_bins > MAX_LDS_BINS) return bad("more than 1024 bins needs a mesh tally");
    if (d->source_kind != MC_SRC_POINT && d->source_kind != MC_SRC_BOX && d->source_kind != MC_SRC_BEAM)
        return bad("unknown source kind");
    if (!(d->source_energy > 0.0) || !(d->energy_cutoff >= 0.0)) return bad("energies must be > 0");
    if (d->source_kind == MC_SRC_BEAM) {
        const double n2 = d->source_dir[0] * d->source_dir[0] + d->source_dir[1] * d->source_dir[1] +
                          d->source_dir[2] * d->source_dir[2];
        if (std::fabs(n2 - 1.0) > 1e-12) return bad("beam direction must be a unit vector");
    }
    g = GeomDev{};
    g.kind = d->kind;
    g.inf_mat = d->material + mat_base;
    g.nx = d->nx;
    g.ny = d->ny;
    g.pitch = d->pitch;
    g.radius = d->radius;
    g.z0 = d->z0;
    g.z1 = d->z1;
    g.mod_mat = d->moderator_material + mat_base;
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
        if (d->tally_kind == MC_TALLY_MESH) g.mesh_h[k] = (g.mesh_hi[k] - g.mesh_lo[k]) / (double)g.mesh_dims[k];
    }
    g.e_cut = d->energy_cutoff;
    int32_t *pm, *lm;
    double *xe, *ee;
    const int32_t zero_i = 0;
    const double zero_d[2] = {0.0, 0.0};
    int rc = MC_OK;
    if (d->kind == MC_GEOM_LATTICE) {
        std::vector<int32_t> pins((size_t)d->nx * d->ny);
        for (size_t c = 0; c < pins.size(); ++c) pins[c] = d->pin_material[c] < 0 ? -1 : d->pin_material[c] + mat_base;
        rc = upload(ctx, B, &pm, pins.data(), pins.size());
    } else {
        rc = upload(ctx, B, &pm, &zero_i, 1);
    }
    if (!rc) {
        if (d->kind == MC_GEOM_SLAB) {
            std::vector<int32_t> lay(d->layer_material, d->layer_material + d->n_layers);
            for (int32_t &m : lay) m += mat_base;
            rc = upload(ctx, B, &xe, d->x_edges, (size_t)d->n_layers + 1);
            if (!rc) rc = upload(ctx, B, &lm, lay.data(), lay.size());
        } else {
            rc = upload(ctx, B, &xe, zero_d, 2);
            if (!rc) rc = upload(ctx, B, &lm, &zero_i, 1);
        }
    }
    if (!rc) {
        if (d->tally_kind == MC_TALLY_ENERGY) rc = upload(ctx, B, &ee, d->energy_edges, (size_t)n_bins + 1);
        else rc = upload(ctx, B, &ee, zero_d, 2);
    }
    if (rc) return rc;
    g.pin_mat = pm;
    g.x_edges = xe;
    g.layer_mat = lm;
    g.e_edges = ee;
    return MC_OK;
}

int mc_init_geometry(mc_ctx *ctx, const mc_geometry_desc *d)
{
    if (!ctx || !d) return MC_EINVAL;
    if (!ctx->have_mat) return fail(ctx, MC_ESTATE, "mc_init_geometry: materials first");
    HIPCHK(hipSetDevice(ctx->device));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->geom_bufs.release();
    ctx->have_geom = false;
    GeomDev g{};
    int rc = build_geometry(ctx, d, ctx->n_mat, 0, ctx->geom_bufs, g, "mc_init_geometry: ");
    const int32_t n_bins = rc ? 0 : g.n_bins;
    for (int t = 0; t < 3 && !rc; ++t) {
        const size_t n = (t == 2) ? (size_t)N_GLOBAL : (size_t)n_bins;
        rc = dalloc(ctx, ctx->geom_bufs, &ctx->S1[t], n);
        if (!rc) rc = dalloc(ctx, ctx->geom_bufs, &ctx->S2[t], n);
    }
    if (rc) {
        ctx->geom_bufs.release();
        return rc;
    }
    ctx->geom = g;
    ctx->n_bins = n_bins;
    ctx->geom_sig = geom_signature(ctx->xs_sig, g);
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
    if (!rc) rc = dalloc(ctx, B, &sb.chunk_off, (chunks + 1) * 256);  // + the digit bases
    if (!rc) HIPCHK(hipMemset(sb.chunk_total, 0, chunks * 256 * sizeof(uint32_t)));
    return rc;
}

// Particle bank of capacity cap and the tally rows of its workgroups.
static int ensure_bank(mc_ctx *ctx, uint32_t cap)
{
    const int32_t chan_bins = ctx->n_chan ? ctx->n_mat * ctx->n_chan : 0;
    if (ctx->cap >= cap && ctx->bank_bins == ctx->n_bins && ctx->tal.n_bins == ctx->n_bins &&
        (ctx->geom.tally_kind == TALLY_MESH) == (ctx->tal.mesh_tl != nullptr) && ctx->tal.n_chan == ctx->n_chan &&
        ctx->tal.chan_bins == chan_bins) {
        ctx->bank.C = cap;  // the first cap slots of the (larger) allocation are in use
        return MC_OK;
    }
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
    if (!rc) rc = dalloc(ctx, B, &b.cp, (size_t)CP_MAX * cap);
    if (!rc && ctx->n_chan) rc = dalloc(ctx, B, &b.sx, (size_t)ctx->n_chan * cap);
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
    if (!rc && mesh) rc = dalloc(ctx, B, &t.mesh_tl, (size_t)ctx->n_bins + 1);    // + underflow count
    if (!rc && mesh) rc = dalloc(ctx, B, &t.mesh_coll, (size_t)ctx->n_bins + 1);
    t.n_chan = ctx->n_chan;
    t.chan_bins = chan_bins;
    if (!rc && chan_bins) rc = dalloc(ctx, B, &t.chan, (size_t)t.rows * (size_t)chan_bins);
    const size_t part_bins = std::max<size_t>(std::max<size_t>(ctx->n_bins, N_GLOBAL), (size_t)chan_bins);
    if (!rc) rc = dalloc(ctx, B, &ctx->partial, (size_t)64 * part_bins);
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

// Split stacks and per-slot importance state for cap slots (only what the
// windows and the estimate configured on the context need).
static int ensure_ww(mc_ctx *ctx, uint32_t cap)
{
    const mc_ww_desc &d = ctx->ww_desc;
    const bool stacks = d.kind != MC_WW_OFF, imp = d.imp_nx > 0;
    if (!stacks && !imp) {
        ctx->ww = WwDev{};
        return MC_OK;
    }
    if (ctx->ww_cap < cap || !ctx->ln_src) {
        HIPCHK(hipStreamSynchronize(ctx->stream));
        ctx->ww_bufs.release();
        ctx->ww_cap = 0;
        Buffers &B = ctx->ww_bufs;
        WwDev w{};
        int rc = dalloc(ctx, B, &ctx->ln_src, 1);
        if (stacks) {
            const size_t nrec = (size_t)d.depth * cap;
            double **dd[] = {&w.sx, &w.sy, &w.sz, &w.su, &w.sv, &w.sw, &w.sE, &w.swt};
            for (double **q : dd)
                if (!rc) rc = dalloc(ctx, B, q, nrec);
            int32_t **ii[] = {&w.scell, &w.smat, &w.sncoll, &w.sncross};
            for (int32_t **q : ii)
                if (!rc) rc = dalloc(ctx, B, q, nrec);
            uint32_t **uu[] = {&w.slin, &w.ssplit, &w.snext, &w.sn};
            for (uint32_t **q : uu)
                if (!rc) rc = dalloc(ctx, B, q, nrec);
            if (!rc) rc = dalloc(ctx, B, &w.sinside, nrec);
            if (!rc) rc = dalloc(ctx, B, &w.sgen, nrec);
            if (!rc) rc = dalloc(ctx, B, &w.depth_of, cap);
            if (!rc) rc = dalloc(ctx, B, &w.splits, cap);
            if (!rc) rc = dalloc(ctx, B, &w.gen, cap);
            if (!rc) rc = dalloc(ctx, B, &w.inh_coll, cap);
            if (!rc) rc = dalloc(ctx, B, &w.inh_cross, cap);
            if (!rc && imp) rc = dalloc(ctx, B, &w.siv, nrec * (size_t)d.imp_ne);
            // copy bank: twice the slots
            const size_t Q = std::max<size_t>((size_t)2 * cap, 256);
            double **qd[] = {&w.qx, &w.qy, &w.qz, &w.qu, &w.qv, &w.qw, &w.qE, &w.qwt};
            for (double **q : qd)
                if (!rc) rc = dalloc(ctx, B, q, Q);
            int32_t **qi[] = {&w.qcell, &w.qmat, &w.qncoll, &w.qncross};
            for (int32_t **q : qi)
                if (!rc) rc = dalloc(ctx, B, q, Q);
            if (!rc) rc = dalloc(ctx, B, &w.qinside, Q);
            if (!rc) rc = dalloc(ctx, B, &w.qgen, Q);
            if (!rc) rc = dalloc(ctx, B, &w.qlin, Q);
            if (!rc) rc = dalloc(ctx, B, &w.qpid, Q);
            if (!rc && imp) rc = dalloc(ctx, B, &w.qiv, Q * (size_t)d.imp_ne);
            w.Q = (uint32_t)Q;
        }
        if (!rc && imp) rc = dalloc(ctx, B, &w.iv, (size_t)cap * (size_t)d.imp_ne);
        if (rc) {
            B.release();
            ctx->ln_src = nullptr;
            return rc;
        }
        ctx->ww = w;
        ctx->ww_cap = cap;
    }
    WwDev &w = ctx->ww;
    w.kind = d.kind;
    w.nmax = d.n_max;
    w.depth = d.depth;
    w.lin0 = d.lin[0];
    w.lin1 = d.lin[1];
    w.lin2 = d.lin[2];
    w.length = d.length;
    w.kappa = d.kappa;
    w.ratio = d.ratio;
    w.ln_emin = std::log(1e-5);
    w.ln_erange = std::log(2e7 / 1e-5);
    w.ln_lo = d.ln_lo;
    w.ln_hi = d.ln_hi;
    w.ln_src = ctx->ln_src;
    w.C = cap;
    w.imp_nx = d.imp_nx;
    w.imp_ne = d.imp_ne;
    w.imp_x0 = d.imp_x0;
    w.imp_x1 = d.imp_x1;
    w.num = ctx->imp_num;
    w.den = ctx->imp_den;
    w.cnt = ctx->imp_cnt;
    if (d.kind == MC_WW_MLP) {
        if (!ctx->have_mlp) return fail(ctx, MC_ESTATE, "weight windows from the network: mc_mlp_set first");
        w.mlp = mlp_dev(ctx);
    }
    if (d.kind != MC_WW_OFF) HIPCHK(launch_ww_source(w, ctx->geom, ctx->ln_src, ctx->stream));
    return MC_OK;
}

// Mesh tallies of one batch: the contributions that fell below the fixed-point
// resolution (the word after the bins of each array), read after the batch.
static int mesh_underflow(mc_ctx *ctx, const TallyDev &t, uint64_t *out)
{
    uint64_t u[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(&u[0], t.mesh_tl + ctx->n_bins, sizeof(uint64_t), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipMemcpyAsync(&u[1], t.mesh_coll + ctx->n_bins, sizeof(uint64_t), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    *out = u[0] + u[1];
    return MC_OK;
}

// Range bound of the fixed-point mesh tallies (see mesh_add): every bin of a
// batch stays below 2^32 T_b + 2^62 units for a batch with weighted track
// total T_b, so T_b < 2^31 rules out a wrapped bin.  T_b is read from the
// global track-length sum the batch added to S1.
static int mesh_range_check(mc_ctx *ctx, uint64_t n)
{
    double s1 = 0.0;
    HIPCHK(hipMemcpyAsync(&s1, ctx->S1[2] + MC_G_TRACK, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    const double Tb = (s1 - ctx->track_s1) * (double)n;
    ctx->track_s1 = s1;
    if (!(Tb < MESH_TRACK_LIMIT))
        return fail(ctx, MC_ERANGE,
                    "mesh tally: the batch's weighted track length " + std::to_string(Tb) +
                        " reaches 2^31, where a fixed-point bin could wrap; reset the tallies and run smaller batches");
    return MC_OK;
}

// One event loop over histories [first_pid, first_pid + n) on the context's
// stream, into the context's own tally rows (view == nullptr) or the rows of
// a view; zero_rows: clear them first; stats: add the batch statistics (and
// count the batch) at the end.
static int run_loop(mc_ctx *ctx, uint64_t seed, uint64_t first_pid, uint64_t n, const mc_run_opts &opts,
                    const TallyDev *view, bool zero_rows, bool stats)
{
    const bool windows = ctx->ww_desc.kind != MC_WW_OFF;
    uint64_t cap64 = opts.in_flight ? opts.in_flight
                                    : (ctx->tune.in_flight > 0 ? (uint64_t)ctx->tune.in_flight
                                                               : (windows ? kDefaultInFlightWindows : kDefaultInFlight));
    // analog: no more slots than histories; with weight windows the copies
    // of split particles take free slots too (up to four per history)
    if (!windows || opts.in_flight) cap64 = std::min(cap64, n);
    else cap64 = std::min(cap64, std::max<uint64_t>(4 * n, 4096));
    if (cap64 > (1ull << 30)) return fail(ctx, MC_EINVAL, "in_flight above 2^30");
    const uint64_t sort_min = opts.sort_min ? opts.sort_min
                                            : (ctx->tune.sort_min > 0 ? (uint64_t)ctx->tune.sort_min : kDefaultSortMin);
    const uint64_t collide_sort_min = ctx->tune.collide_sort_min > 0 ? (uint64_t)ctx->tune.collide_sort_min : sort_min;
    const int64_t max_events = opts.max_events > 0 ? opts.max_events : kDefaultMaxEvents;
    HistLog *log = static_cast<HistLog *>(opts.history_log);
    const uint32_t cap = (uint32_t)cap64;
    int rc = ensure_bank(ctx, cap);
    if (!rc) rc = ensure_ww(ctx, cap);
    if (rc) return rc;
    hipStream_t st = ctx->stream;
    BankDev &b = ctx->bank;
    const WwDev &W = ctx->ww;
    TallyDev tal = view ? *view : ctx->tal;
    tal.enabled = opts.no_tally ? 0 : 1;
    const GeomDev &g = ctx->geom;
    const bool mesh = g.tally_kind == TALLY_MESH;

    // reset per-batch state
    HIPCHK(launch_fill_u8(b.flags, cap, 0, st));
    const size_t row_bins = mesh ? 1 : (size_t)ctx->n_bins;
    if (zero_rows) {
        HIPCHK(launch_fill_f64(tal.tl, (size_t)tal.rows * row_bins, 0.0, st));
        HIPCHK(launch_fill_f64(tal.coll, (size_t)tal.rows * row_bins, 0.0, st));
        HIPCHK(launch_fill_f64(tal.glob, (size_t)tal.rows * N_GLOBAL, 0.0, st));
        if (tal.chan) HIPCHK(launch_fill_f64(tal.chan, (size_t)tal.rows * (size_t)tal.chan_bins, 0.0, st));
        if (mesh) {
            HIPCHK(launch_fill_f64(tal.mesh_tl, (size_t)ctx->n_bins + 1, 0.0, st));
            HIPCHK(launch_fill_f64(tal.mesh_coll, (size_t)ctx->n_bins + 1, 0.0, st));
        }
    }
    HIPCHK(launch_fill_u32(reinterpret_cast<uint32_t *>(ctx->ctr), 2 * sizeof(Counters) / 4, 0u, st));
    // with windows, copies add into their history's record: it starts zeroed
    if (log && W.kind != WW_OFF) HIPCHK(launch_fill_u32(reinterpret_cast<uint32_t *>(log), n * sizeof(HistLog) / 4, 0u, st));
    // every slot's stack starts empty (the flush reads the depth of all slots,
    // also of slots that never held a particle)
    if (W.kind != WW_OFF) HIPCHK(launch_fill_u8(W.depth_of, cap, 0, st));
    HIPCHK(launch_fill_u32(reinterpret_cast<uint32_t *>(ctx->dstat), 8, 0u, st));

    mc_stats s{};
    size_t n_timed = 0;
    // with time_kernels: the kind of each timed launch (event pair n_timed)
    enum { T_LOOKUP = 0, T_ADVANCE = 1, T_CROSS = 2, T_COLLIDE = 3 };
    std::vector<int> timed_kind;
    auto time_begin = [&](int kind) -> int {
        if (!opts.time_kernels) return MC_OK;
        int r = timing_event_pair(ctx, n_timed);
        if (r) return r;
        timed_kind.push_back(kind);
        HIPCHK(hipEventRecord(ctx->ev_a[n_timed], st));
        return MC_OK;
    };
    auto time_end = [&]() -> int {
        if (!opts.time_kernels) return MC_OK;
        HIPCHK(hipEventRecord(ctx->ev_b[n_timed], st));
        ++n_timed;
        return MC_OK;
    };
    // the timed launches' durations, summed per kind into s
    auto sum_timed = [&]() -> int {
        for (size_t k = 0; k < n_timed; ++k) {
            float t = 0.f;
            HIPCHK(hipEventElapsedTime(&t, ctx->ev_a[k], ctx->ev_b[k]));
            switch (timed_kind[k]) {
            case T_LOOKUP: s.lookup_ms += t; break;
            case T_ADVANCE: s.advance_ms += t; break;
            case T_CROSS: s.cross_ms += t; break;
            default: s.collide_ms += t; break;
            }
        }
        return MC_OK;
    };
    HIPCHK(hipEventRecord(ctx->ev_batch0, st));
    uint64_t it = 0;
    // every history ends within max_events + 1 iterations of its start, so the
    // loop is bounded by the number of bank refills times that
    // (with weight windows a history also runs its pending copies one by one)
    uint64_t max_iter = (n / cap + 2) * ((uint64_t)max_events + 2);
    if (W.kind != WW_OFF) max_iter *= 1ull + (uint64_t)W.depth * (uint64_t)W.nmax;
    // The host runs one iteration behind the GPU: after the first iteration
    // (whose queue lengths it waits for) it queues iteration `it` while the
    // GPU still works on iteration it - 1, knowing the queue lengths of
    // it - 1 only (copied to the host as soon as that iteration's queues were
    // built).  Every kernel reads its exact length from the device counters;
    // the host sizes grids by bounds: with no histories left to start and no
    // weight-window copies, no queue grows, so iteration it's queues are no
    // longer than it - 1's alive queue, and otherwise the bank capacity
    // bounds them.  Its choices (sort or not, the one-launch tail) follow
    // it - 1's lengths, which changes no result: a sorted queue only reorders
    // the lookups, and the tail runs the same histories.  The loop ends when
    // it - 1 had no particle alive (one empty iteration queued).
    Counters p{};                 // lengths of iteration it - 1 (of it itself when it = 0)
    bool sorted_prev = false;     // iteration it - 1 sorted its lookup queue
    bool tail_run = false;
    const bool analog = W.kind == WW_OFF;
    for (;; ++it) {
        if (it >= max_iter) return fail(ctx, MC_EHIP, "event loop did not terminate");
        const int cur = (int)(it & 1);
        const bool exact = it == 0;
        if (!exact) {  // the lengths of iteration it - 1 (its queues were built long ago)
            HIPCHK(hipEventSynchronize(ctx->ev_ctr[cur ^ 1]));
            p = ctx->ctr_host[cur ^ 1];
            s.lookups += p.nL;
            if (sorted_prev) s.sorted_lookups += p.nL;
            s.flights += p.nA;
            if (p.nA == 0) {  // iteration it - 1 was empty: every history ended before it
                if (p.issued != n || p.top != 0)
                    return fail(ctx, MC_EHIP, "event loop ended before every history (and copy) was run");
                --it;  // iterations with particles: 0 .. it - 2
                break;
            }
        }
        HIPCHK(launch_slots_count(b, st));
        const uint32_t new_bound = (uint32_t)std::min<uint64_t>(cap, n - p.issued);  // histories not yet started
        HIPCHK(launch_slots_queue(b, g, W, ctx->ctr, cur, first_pid, n, seed, new_bound, st));
        HIPCHK(hipMemcpyAsync(ctx->ctr_host + cur, ctx->ctr + cur, sizeof(Counters), hipMemcpyDeviceToHost, st));
        HIPCHK(hipEventRecord(ctx->ev_ctr[cur], st));
        if (exact) {
            HIPCHK(hipEventSynchronize(ctx->ev_ctr[cur]));
            p = ctx->ctr_host[cur];
            if (p.nA == 0) {
                if (p.issued != n || p.top != 0)
                    return fail(ctx, MC_EHIP, "event loop ended before every history (and copy) was run");
                break;
            }
        }
        Counters *dc = ctx->ctr + cur;
        const uint32_t bound = (exact || (analog && p.issued == n)) ? p.nA : cap;
        const int64_t tail = tail_particles(ctx);
        if (tail > 0 && analog && W.imp_nx == 0 && p.issued == n && (int64_t)p.nA <= tail) {
            // every history has started and few remain: finish them in one launch
            HIPCHK(launch_tail(b, ctx->xs, g, tal, dc, bound, seed, max_events, log, first_pid, ctx->dstat + 1, st));
            tail_run = true;
            ++it;
            break;
        }
        {
            LookupLaunch l;
            l.xs = ctx->xs;
            l.n_ptr = &dc->nL;
            l.n_bound = bound;
            l.E = b.E;
            l.mat = b.mat;
            l.Sa = b.Sa;
            l.Ss = b.Ss;
            l.flags = b.flags;
            l.nuc_count = ctx->dstat;
            l.ilp = lookup_ilp(ctx);
            l.cp = b.cp;
            l.sx = b.sx;
            sorted_prev = (uint64_t)p.nL >= sort_min && sort_min != UINT64_MAX;
            if (sorted_prev) {
                HIPCHK(launch_sort(ctx->xs, b.L, &dc->nL, bound, b.E, b.mat, ctx->bank_sort, ctx->n_keys, b.Ls,
                                   b.Lkey, st));
                l.list = b.Ls;
                l.keys = b.Lkey;
            } else {
                l.list = b.L;
            }
            if ((rc = time_begin(T_LOOKUP))) return rc;
            HIPCHK(launch_lookup(l, st));
            if ((rc = time_end())) return rc;
            s.lookup_launches += 1;
        }
        // analog runs without an importance grid cross surfaces in the flight
        // kernel (the split then queues only collisions)
        const bool fuse_cross = analog && W.imp_nx == 0;
        if ((rc = time_begin(T_ADVANCE))) return rc;
        HIPCHK(launch_advance(b, g, tal, W, dc, bound, seed, max_events, log ? 1 : 0, fuse_cross, log, first_pid,
                              ctx->dstat + 1, st));
        if ((rc = time_end())) return rc;
        if ((rc = time_begin(T_CROSS))) return rc;
        HIPCHK(launch_split(b, dc, bound, st));
        if (!fuse_cross) HIPCHK(launch_cross(b, g, tal, W, dc, bound, seed, log, first_pid, ctx->dstat + 1, st));
        if ((rc = time_end())) return rc;
        if ((rc = time_begin(T_COLLIDE))) return rc;
        // collisions re-gather sigma_s: in (material, energy) order when the
        // queues are long enough to sort (the sorted lookup queue is no longer
        // needed, its buffers take the sorted collide queue)
        const uint32_t *qc = b.Qc;
        if ((uint64_t)p.nA >= collide_sort_min && collide_sort_min != UINT64_MAX) {
            HIPCHK(launch_sort(ctx->xs, b.Qc, &dc->nC, bound, b.E, b.mat, ctx->bank_sort, ctx->n_keys, b.Ls, b.Lkey,
                               st));
            qc = b.Ls;
        }
        HIPCHK(launch_collide(b, qc, ctx->xs, g, tal, W, dc, bound, seed, log, first_pid, st));
        if ((rc = time_end())) return rc;
        if (W.kind != WW_OFF) HIPCHK(launch_ww_flush(b, W, dc, st));
    }
    if (tail_run) {  // the tail's particle count: the lengths of its iteration
        HIPCHK(hipStreamSynchronize(st));
        s.tail_particles = ctx->ctr_host[(it - 1) & 1].nA;
    }
    if (!stats) {  // a worker of concurrent loops or batches: its caller forms the statistics
        HIPCHK(hipEventRecord(ctx->ev_batch1, st));
        unsigned long long dstat[2] = {0, 0};
        HIPCHK(hipMemcpyAsync(dstat, ctx->dstat, sizeof(dstat), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if ((rc = sum_timed())) return rc;
        s.iterations = it;
        s.nuclide_lookups = dstat[0];
        s.lost = dstat[1];
        if (mesh && !view) {  // own mesh arrays (with a view the caller reads the shared ones)
            rc = mesh_underflow(ctx, tal, &s.mesh_underflow);
            if (rc) return rc;
        }
        ctx->stats = s;
        return MC_OK;
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
    if (tal.chan)
        HIPCHK(launch_batch_stats(tal.chan, tal.rows, tal.chan_bins, nullptr, ctx->partial, inv_n, ctx->S1[3],
                                  ctx->S2[3], st));
    HIPCHK(hipEventRecord(ctx->ev_batch1, st));
    unsigned long long dstat[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(dstat, ctx->dstat, sizeof(dstat), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, ctx->ev_batch0, ctx->ev_batch1));
    s.batch_ms = ms;
    if ((rc = sum_timed())) return rc;
    s.iterations = it;
    s.nuclide_lookups = dstat[0];
    s.lost = dstat[1];
    // per lookup 36 B (+ 8 B per channel written), per nuclide 56 B (+ 16 B per channel)
    s.lookup_bytes = (36ull + 8ull * (uint64_t)ctx->n_chan) * s.lookups +
                     (56ull + 16ull * (uint64_t)ctx->n_chan) * s.nuclide_lookups;
    if (mesh) {
        rc = mesh_underflow(ctx, tal, &s.mesh_underflow);
        if (rc) return rc;
    }
    ctx->stats = s;
    ctx->n_batches += 1;
    ctx->histories += n;
    if (mesh) {
        rc = mesh_range_check(ctx, n);
        if (rc) return rc;
    }
    if (s.lost > opts.max_lost)
        return fail(ctx, MC_ELOST, std::to_string(s.lost) + " particles lost (event cap reached)");
    return MC_OK;
}

// Worker contexts of concurrent loops: own stream (default priority), bank,
// counters and events; the tables and tallies of ctx, refreshed per batch.
static int ensure_workers(mc_ctx *ctx, int L)
{
    while ((int)ctx->workers.size() < L) {
        hipStream_t st = nullptr;
        HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        mc_ctx *w = nullptr;
        const int rc = mc_create(&w, ctx->device, st, ctx->has_alloc ? &ctx->alloc : nullptr);
        if (rc) {
            (void)hipStreamDestroy(st);
            return fail(ctx, rc, "concurrent loops: worker context");
        }
        w->owns_stream = true;
        ctx->workers.push_back(w);
        hipEvent_t e = nullptr;
        HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        ctx->ev_loop_done.push_back(e);
    }
    if (!ctx->ev_loop_start) HIPCHK(hipEventCreateWithFlags(&ctx->ev_loop_start, hipEventDisableTiming));
    for (int l = 0; l < L; ++l) {
        mc_ctx *w = ctx->workers[l];
        w->have_mat = w->have_geom = true;
        w->xs = ctx->xs;
        w->geom = ctx->geom;
        w->n_bins = ctx->n_bins;
        w->n_mat = ctx->n_mat;
        w->n_nuc = ctx->n_nuc;
        w->n_keys = ctx->n_keys;
        w->n_chan = ctx->n_chan;
        w->tune = ctx->tune;
        w->tune.loops = 1;
        w->ww_desc = mc_ww_desc{};
        w->ww_desc.kind = MC_WW_OFF;
    }
    return MC_OK;
}

// Tally rows of L concurrent loops of R rows each (and the shared mesh
// arrays), laid out so that the batch statistics read them as one array.
static int ensure_loop_rows(mc_ctx *ctx, int L, int32_t R)
{
    const bool mesh = ctx->geom.tally_kind == TALLY_MESH;
    const int32_t chan_bins = ctx->n_chan ? ctx->n_mat * ctx->n_chan : 0;
    if (ctx->loop_n == L && ctx->loop_rows >= R && ctx->loop_bins == ctx->n_bins && ctx->loop_mesh == mesh &&
        ctx->loop_chan_bins == chan_bins)
        return MC_OK;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->loop_bufs.release();
    ctx->loop_n = 0;
    Buffers &B = ctx->loop_bufs;
    TallyDev t{};
    t.n_bins = ctx->n_bins;
    t.rows = L * R;
    t.n_chan = ctx->n_chan;
    t.chan_bins = chan_bins;
    const size_t row_bins = mesh ? 1 : (size_t)ctx->n_bins;
    int rc = dalloc(ctx, B, &t.tl, (size_t)t.rows * row_bins);
    if (!rc) rc = dalloc(ctx, B, &t.coll, (size_t)t.rows * row_bins);
    if (!rc) rc = dalloc(ctx, B, &t.glob, (size_t)t.rows * N_GLOBAL);
    if (!rc && mesh) rc = dalloc(ctx, B, &t.mesh_tl, (size_t)ctx->n_bins + 1);    // + underflow count
    if (!rc && mesh) rc = dalloc(ctx, B, &t.mesh_coll, (size_t)ctx->n_bins + 1);
    if (!rc && chan_bins) rc = dalloc(ctx, B, &t.chan, (size_t)t.rows * (size_t)chan_bins);
    const size_t part_bins = std::max<size_t>(std::max<size_t>(ctx->n_bins, N_GLOBAL), (size_t)chan_bins);
    if (!rc) rc = dalloc(ctx, B, &ctx->loop_partial, (size_t)64 * part_bins);
    if (rc) {
        B.release();
        return rc;
    }
    ctx->loop_tal = t;
    ctx->loop_n = L;
    ctx->loop_rows = R;
    ctx->loop_bins = ctx->n_bins;
    ctx->loop_mesh = mesh;
    ctx->loop_chan_bins = chan_bins;
    return MC_OK;
}

// L event loops at once (the paper runs several ranks per GPU for the same
// effect): loop l takes the l-th contiguous share of the pids on its own
// stream, driven by its own host thread; the batch statistics sum the rows of
// loop 0, then loop 1, ... (fixed order: reruns are bitwise identical).
static int run_concurrent(mc_ctx *ctx, int L, uint64_t seed, uint64_t first_pid, uint64_t n,
                          const mc_run_opts &opts)
{
    int rc = ensure_workers(ctx, L);
    if (rc) return rc;
    const uint64_t per_max = (n + (uint64_t)L - 1) / (uint64_t)L;
    uint64_t cap = opts.in_flight ? opts.in_flight
                                  : (ctx->tune.in_flight > 0 ? (uint64_t)ctx->tune.in_flight : kDefaultInFlight);
    cap = std::min(cap, per_max);
    if (cap > (1ull << 30)) return fail(ctx, MC_EINVAL, "in_flight above 2^30");
    const int32_t R = (int32_t)((cap + WG - 1) / WG);
    rc = ensure_loop_rows(ctx, L, R);
    if (rc) return rc;
    hipStream_t st = ctx->stream;
    const bool mesh = ctx->geom.tally_kind == TALLY_MESH;
    TallyDev all = ctx->loop_tal;
    all.enabled = opts.no_tally ? 0 : 1;
    const size_t row_bins = mesh ? 1 : (size_t)ctx->n_bins;
    HIPCHK(hipEventRecord(ctx->ev_batch0, st));
    HIPCHK(launch_fill_f64(all.tl, (size_t)all.rows * row_bins, 0.0, st));
    HIPCHK(launch_fill_f64(all.coll, (size_t)all.rows * row_bins, 0.0, st));
    HIPCHK(launch_fill_f64(all.glob, (size_t)all.rows * N_GLOBAL, 0.0, st));
    if (all.chan) HIPCHK(launch_fill_f64(all.chan, (size_t)all.rows * (size_t)all.chan_bins, 0.0, st));
    if (mesh) {
        HIPCHK(launch_fill_f64(all.mesh_tl, (size_t)ctx->n_bins + 1, 0.0, st));
        HIPCHK(launch_fill_f64(all.mesh_coll, (size_t)ctx->n_bins + 1, 0.0, st));
    }
    HIPCHK(hipEventRecord(ctx->ev_loop_start, st));
    std::vector<TallyDev> views(L);
    std::vector<mc_run_opts> wopts(L, opts);
    std::vector<uint64_t> first(L), count(L);
    uint64_t next = first_pid;
    for (int l = 0; l < L; ++l) {
        count[l] = n / (uint64_t)L + ((uint64_t)l < n % (uint64_t)L ? 1 : 0);
        first[l] = next;
        next += count[l];
        TallyDev v = all;
        v.rows = R;
        v.tl = all.tl + (size_t)l * R * row_bins;
        v.coll = all.coll + (size_t)l * R * row_bins;
        v.glob = all.glob + (size_t)l * R * N_GLOBAL;
        if (all.chan) v.chan = all.chan + (size_t)l * R * (size_t)all.chan_bins;
        views[l] = v;
        wopts[l].in_flight = std::min<uint64_t>(cap, count[l]);
        wopts[l].max_lost = UINT64_MAX;  // counted over all loops below
        if (opts.history_log)
            wopts[l].history_log = static_cast<HistLog *>(opts.history_log) + (first[l] - first_pid);
        HIPCHK(hipStreamWaitEvent(ctx->workers[l]->stream, ctx->ev_loop_start, 0));
    }
    std::vector<int> wrc(L, MC_OK);
    auto body = [&](int l) {
        mc_ctx *w = ctx->workers[l];
        if (hipSetDevice(w->device) != hipSuccess) {
            wrc[l] = fail(w, MC_EHIP, "hipSetDevice");
            return;
        }
        wrc[l] = run_loop(w, seed, first[l], count[l], wopts[l], &views[l], false, false);
    };
    std::vector<std::thread> threads;
    for (int l = 1; l < L; ++l) threads.emplace_back(body, l);
    body(0);
    for (std::thread &t : threads) t.join();
    for (int l = 0; l < L; ++l) {
        if (wrc[l]) {
            HIPCHK(hipDeviceSynchronize());
            return fail(ctx, wrc[l], "concurrent loop " + std::to_string(l) + ": " + ctx->workers[l]->err);
        }
    }
    for (int l = 0; l < L; ++l) {
        HIPCHK(hipEventRecord(ctx->ev_loop_done[l], ctx->workers[l]->stream));
        HIPCHK(hipStreamWaitEvent(st, ctx->ev_loop_done[l], 0));
    }
    const double inv_n = 1.0 / (double)n;
    double *part = ctx->loop_partial;
    if (mesh) {
        HIPCHK(launch_batch_stats(nullptr, 0, ctx->n_bins, all.mesh_tl, part, inv_n, ctx->S1[0], ctx->S2[0], st));
        HIPCHK(launch_batch_stats(nullptr, 0, ctx->n_bins, all.mesh_coll, part, inv_n, ctx->S1[1], ctx->S2[1], st));
    } else {
        HIPCHK(launch_batch_stats(all.tl, all.rows, ctx->n_bins, nullptr, part, inv_n, ctx->S1[0], ctx->S2[0], st));
        HIPCHK(launch_batch_stats(all.coll, all.rows, ctx->n_bins, nullptr, part, inv_n, ctx->S1[1], ctx->S2[1], st));
    }
    HIPCHK(launch_batch_stats(all.glob, all.rows, N_GLOBAL, nullptr, part, inv_n, ctx->S1[2], ctx->S2[2], st));
    if (all.chan)
        HIPCHK(launch_batch_stats(all.chan, all.rows, all.chan_bins, nullptr, part, inv_n, ctx->S1[3], ctx->S2[3],
                                  st));
    HIPCHK(hipEventRecord(ctx->ev_batch1, st));
    HIPCHK(hipStreamSynchronize(st));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, ctx->ev_batch0, ctx->ev_batch1));
    mc_stats s{};
    for (int l = 0; l < L; ++l) {
        const mc_stats &q = ctx->workers[l]->stats;
        add_stats(s, q);
        s.mesh_underflow = 0;  // counted once below from the shared mesh arrays
        s.iterations = std::max(s.iterations, q.iterations);
    }
    s.batch_ms = ms;
    s.lookup_bytes = (36ull + 8ull * (uint64_t)ctx->n_chan) * s.lookups +
                     (56ull + 16ull * (uint64_t)ctx->n_chan) * s.nuclide_lookups;
    if (mesh) {
        rc = mesh_underflow(ctx, all, &s.mesh_underflow);
        if (rc) return rc;
    }
    ctx->stats = s;
    ctx->n_batches += 1;
    ctx->histories += n;
    if (mesh) {
        rc = mesh_range_check(ctx, n);
        if (rc) return rc;
    }
    if (s.lost > opts.max_lost)
        return fail(ctx, MC_ELOST, std::to_string(s.lost) + " particles lost (event cap reached)");
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
    // concurrent loops: analog batches of at least 4096 histories per loop
    int L = ctx->tune.loops > 1 ? ctx->tune.loops : 1;
    if (ctx->ww_desc.kind != MC_WW_OFF || ctx->ww_desc.imp_nx > 0) L = 1;
    while (L > 1 && n / (uint64_t)L < 4096) --L;
    if (L > 1) return run_concurrent(ctx, L, seed, first_pid, n, opts);
    return run_loop(ctx, seed, first_pid, n, opts, nullptr, true, true);
}

// Batches b = 0 .. n_batches-1 of pids [first_pid + b n, first_pid + (b+1) n),
// up to `loops` of them at once, each whole batch on one worker (its own
// stream, bank and rows; the next batch goes to the first worker free).
// Every batch's value is formed from its own rows exactly as mc_run_batch
// forms it, and the statistics take the values in batch order: the tallies
// equal those of n_batches mc_run_batch calls bit for bit.
int mc_run_batches(mc_ctx *ctx, uint64_t seed, uint64_t first_pid, uint64_t n, uint64_t n_batches,
                   const mc_run_opts *opts_in)
{
    if (!ctx) return MC_EINVAL;
    if (!ctx->have_geom) return fail(ctx, MC_ESTATE, "mc_run_batches: materials and geometry first");
    if (n == 0 || n_batches == 0) return fail(ctx, MC_EINVAL, "mc_run_batches: n and n_batches must be >= 1");
    if (n_batches > (1u << 20)) return fail(ctx, MC_EINVAL, "mc_run_batches: at most 2^20 batches per call");
    HIPCHK(hipSetDevice(ctx->device));
    mc_run_opts opts{};
    if (opts_in) opts = *opts_in;
    int L = ctx->tune.loops > 1 ? ctx->tune.loops : 1;
    if (ctx->ww_desc.kind != MC_WW_OFF || ctx->ww_desc.imp_nx > 0) L = 1;
    if ((uint64_t)L > n_batches) L = (int)n_batches;
    if (L <= 1) {
        mc_stats tot{};
        const auto t0 = std::chrono::steady_clock::now();
        for (uint64_t b = 0; b < n_batches; ++b) {
            mc_run_opts o = opts;
            if (opts.history_log) o.history_log = static_cast<HistLog *>(opts.history_log) + b * n;
            const int rc = mc_run_batch(ctx, seed, first_pid + b * n, n, &o);
            if (rc) return rc;
            const mc_stats &q = ctx->stats;
            tot.iterations += q.iterations;
            tot.lookup_bytes += q.lookup_bytes;
            add_stats(tot, q);
        }
        tot.batch_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        ctx->stats = tot;
        return MC_OK;
    }
    int rc = ensure_workers(ctx, L);
    if (rc) return rc;
    const bool mesh = ctx->geom.tally_kind == TALLY_MESH;
    const int32_t nb_t = ctx->n_bins, nb_r = ctx->n_chan ? ctx->n_mat * ctx->n_chan : 0;
    const size_t cols = 2 * (size_t)nb_t + N_GLOBAL + (size_t)nb_r;  // tl, coll, glob, reaction
    if (ctx->batch_vals_n < n_batches * cols) {
        HIPCHK(hipStreamSynchronize(ctx->stream));
        ctx->batch_bufs.release();
        ctx->batch_vals_n = 0;
        rc = dalloc(ctx, ctx->batch_bufs, &ctx->batch_vals, n_batches * cols);
        if (rc) return rc;
        ctx->batch_vals_n = n_batches * cols;
    }
    hipStream_t st = ctx->stream;
    HIPCHK(hipEventRecord(ctx->ev_batch0, st));
    HIPCHK(hipEventRecord(ctx->ev_loop_start, st));
    for (int l = 0; l < L; ++l) HIPCHK(hipStreamWaitEvent(ctx->workers[l]->stream, ctx->ev_loop_start, 0));
    std::atomic<uint64_t> next{0};
    std::atomic<bool> failed{false};
    std::vector<int> wrc(L, MC_OK);
    std::vector<mc_stats> tot(L);
    const double inv_n = 1.0 / (double)n;
    auto body = [&](int l) {
        mc_ctx *w = ctx->workers[l];
        if (hipSetDevice(w->device) != hipSuccess) {
            wrc[l] = fail(w, MC_EHIP, "hipSetDevice");
            failed = true;
            return;
        }
        for (;;) {
            const uint64_t b = next++;
            if (b >= n_batches || failed) return;
            mc_run_opts o = opts;
            o.max_lost = UINT64_MAX;  // counted over all batches below
            if (opts.history_log) o.history_log = static_cast<HistLog *>(opts.history_log) + b * n;
            int r = run_loop(w, seed, first_pid + b * n, n, o, nullptr, true, false);
            // the batch's value from its rows, as mc_run_batch forms it
            const TallyDev &t = w->tal;
            double *T = ctx->batch_vals + b * cols;
            hipStream_t ws = w->stream;
            if (!r) {
                hipError_t e = hipSuccess;
                if (mesh) {
                    e = launch_batch_stats(nullptr, 0, nb_t, t.mesh_tl, w->partial, inv_n, T, nullptr, ws);
                    if (e == hipSuccess)
                        e = launch_batch_stats(nullptr, 0, nb_t, t.mesh_coll, w->partial, inv_n, T + nb_t, nullptr, ws);
                } else {
                    e = launch_batch_stats(t.tl, t.rows, nb_t, nullptr, w->partial, inv_n, T, nullptr, ws);
                    if (e == hipSuccess)
                        e = launch_batch_stats(t.coll, t.rows, nb_t, nullptr, w->partial, inv_n, T + nb_t, nullptr, ws);
                }
                if (e == hipSuccess)
                    e = launch_batch_stats(t.glob, t.rows, N_GLOBAL, nullptr, w->partial, inv_n, T + 2 * nb_t,
                                           nullptr, ws);
                if (e == hipSuccess && t.chan)
                    e = launch_batch_stats(t.chan, t.rows, nb_r, nullptr, w->partial, inv_n,
                                           T + 2 * nb_t + N_GLOBAL, nullptr, ws);
                if (e != hipSuccess) r = fail(w, MC_EHIP, hipGetErrorString(e));
            }
            if (r) {
                wrc[l] = r;
                failed = true;
                return;
            }
            const mc_stats &q = w->stats;
            mc_stats &a = tot[l];
            a.iterations += q.iterations;
            add_stats(a, q);
        }
    };
    std::vector<std::thread> threads;
    for (int l = 1; l < L; ++l) threads.emplace_back(body, l);
    body(0);
    for (std::thread &t : threads) t.join();
    for (int l = 0; l < L; ++l) {
        if (wrc[l]) {
            HIPCHK(hipDeviceSynchronize());
            return fail(ctx, wrc[l], "concurrent batches, loop " + std::to_string(l) + ": " + ctx->workers[l]->err);
        }
    }
    for (int l = 0; l < L; ++l) {
        HIPCHK(hipEventRecord(ctx->ev_loop_done[l], ctx->workers[l]->stream));
        HIPCHK(hipStreamWaitEvent(st, ctx->ev_loop_done[l], 0));
    }
    // the statistics, batch by batch in order (columns of one tally are
    // contiguous in every batch's value row: accumulate per tally)
    const int32_t nbk = (int32_t)n_batches;
    const double *V = ctx->batch_vals;
    // values are rows of `cols`; gather each tally's columns with its stride
    HIPCHK(launch_batch_accum_strided(V, nbk, (int32_t)cols, 0, nb_t, ctx->S1[0], ctx->S2[0], st));
    HIPCHK(launch_batch_accum_strided(V, nbk, (int32_t)cols, nb_t, nb_t, ctx->S1[1], ctx->S2[1], st));
    HIPCHK(launch_batch_accum_strided(V, nbk, (int32_t)cols, 2 * nb_t, N_GLOBAL, ctx->S1[2], ctx->S2[2], st));
    if (nb_r)
        HIPCHK(launch_batch_accum_strided(V, nbk, (int32_t)cols, 2 * nb_t + N_GLOBAL, nb_r, ctx->S1[3], ctx->S2[3],
                                          st));
    HIPCHK(hipEventRecord(ctx->ev_batch1, st));
    HIPCHK(hipStreamSynchronize(st));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, ctx->ev_batch0, ctx->ev_batch1));
    mc_stats s{};
    for (const mc_stats &a : tot) {
        s.iterations += a.iterations;
        add_stats(s, a);
    }
    s.batch_ms = ms;
    s.lookup_bytes = (36ull + 8ull * (uint64_t)ctx->n_chan) * s.lookups +
                     (56ull + 16ull * (uint64_t)ctx->n_chan) * s.nuclide_lookups;
    ctx->stats = s;
    ctx->n_batches += n_batches;
    ctx->histories += n * n_batches;
    if (mesh) {
        // every batch's weighted track total (its per-source value times n)
        std::vector<double> tb(n_batches);
        HIPCHK(hipMemcpy2DAsync(tb.data(), sizeof(double), ctx->batch_vals + 2 * (size_t)nb_t + MC_G_TRACK,
                                cols * sizeof(double), sizeof(double), n_batches, hipMemcpyDeviceToHost, st));
        double s1 = 0.0;
        HIPCHK(hipMemcpyAsync(&s1, ctx->S1[2] + MC_G_TRACK, sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        ctx->track_s1 = s1;
        for (uint64_t b = 0; b < n_batches; ++b)
            if (!(tb[b] * (double)n < MESH_TRACK_LIMIT))
                return fail(ctx, MC_ERANGE,
                            "mesh tally: batch " + std::to_string(b) + "'s weighted track length reaches 2^31, "
                            "where a fixed-point bin could wrap; reset the tallies and run smaller batches");
    }
    if (s.lost > opts.max_lost)
        return fail(ctx, MC_ELOST, std::to_string(s.lost) + " particles lost (event cap reached)");
    return MC_OK;
}

int mc_get_tallies(mc_ctx *ctx, int32_t tally_id, double *mean, double *stderr_, size_t n_bins,
                   mc_tally_meta *meta)
{
    if (!ctx) return MC_EINVAL;
    if (!ctx->have_geom) return fail(ctx, MC_ESTATE, "no geometry");
    if (tally_id < 0 || tally_id > 3) return fail(ctx, MC_EINVAL, "unknown tally id");
    if (tally_id == MC_T_REACTION && !ctx->n_chan) return fail(ctx, MC_ESTATE, "no reaction channels");
    const size_t nb = (tally_id == MC_T_GLOBAL)     ? (size_t)N_GLOBAL
                      : (tally_id == MC_T_REACTION) ? (size_t)ctx->n_mat * (size_t)ctx->n_chan
                                                    : (size_t)ctx->n_bins;
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
        if (meta->s1) std::memcpy(meta->s1, s1.data(), nb * sizeof(double));
        if (meta->s2) std::memcpy(meta->s2, s2.data(), nb * sizeof(double));
    }
    return MC_OK;
}

int mc_set_tallies(mc_ctx *ctx, int32_t tally_id, const double *s1, const double *s2, size_t n_bins,
                   uint64_t n_batches, uint64_t histories)
{
    if (!ctx) return MC_EINVAL;
    if (!ctx->have_geom) return fail(ctx, MC_ESTATE, "no geometry");
    if (tally_id < 0 || tally_id > 3) return fail(ctx, MC_EINVAL, "unknown tally id");
    if (tally_id == MC_T_REACTION && !ctx->n_chan) return fail(ctx, MC_ESTATE, "no reaction channels");
    if (!s1 || !s2) return fail(ctx, MC_EINVAL, "mc_set_tallies: s1 and s2 are required");
    const size_t nb = (tally_id == MC_T_GLOBAL)     ? (size_t)N_GLOBAL
                      : (tally_id == MC_T_REACTION) ? (size_t)ctx->n_mat * (size_t)ctx->n_chan
                                                    : (size_t)ctx->n_bins;
    if (n_bins != nb) return fail(ctx, MC_EINVAL, "n_bins does not match the tally (" + std::to_string(nb) + ")");
    if (histories < n_batches) return fail(ctx, MC_EINVAL, "mc_set_tallies: fewer histories than batches");
    for (size_t k = 0; k < nb; ++k)
        if (!std::isfinite(s1[k]) || !std::isfinite(s2[k]) || s2[k] < 0.0)
            return fail(ctx, MC_EINVAL, "mc_set_tallies: bin " + std::to_string(k) + " is not a valid sum");
    HIPCHK(hipSetDevice(ctx->device));
    HIPCHK(hipMemcpyAsync(ctx->S1[tally_id], s1, nb * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(ctx->S2[tally_id], s2, nb * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->n_batches = n_batches;
    ctx->histories = histories;
    if (tally_id == MC_T_GLOBAL) ctx->track_s1 = s1[MC_G_TRACK];
    return MC_OK;
}

int mc_ww_bootstrap_slope(mc_ctx *ctx, double *slope)
{
    if (!ctx || !slope) return MC_EINVAL;
    if (!ctx->have_geom) return fail(ctx, MC_ESTATE, "no geometry");
    if (ctx->n_batches == 0 || ctx->histories == 0) return fail(ctx, MC_ESTATE, "mc_ww_bootstrap_slope: no batch run");
    double mean[N_GLOBAL];
    const int rc = mc_get_tallies(ctx, MC_T_GLOBAL, mean, nullptr, N_GLOBAL, nullptr);
    if (rc) return rc;
    // the far face's importance relative to the source: the pilot's response,
    // floored at one history in the pilot when none scored
    const double r0 = std::max(mean[MC_G_LEAK_XHI], 1.0 / (double)ctx->histories);
    *slope = -std::log(r0);
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
    if (t->sort_min < 0 || t->in_flight < 0 || t->set_grid < 0 || t->collide_sort_min < 0)
        return fail(ctx, MC_EINVAL, "negative tuning value");
    if (t->loops < 0 || t->loops > 8) return fail(ctx, MC_EINVAL, "loops must be in [0, 8]");
    if (t->set_tile_histories < 0 || t->set_tile_histories % WG != 0)
        return fail(ctx, MC_EINVAL, "set_tile_histories must be a multiple of 256");
    ctx->tune = *t;
    return MC_OK;
}

int mc_get_tuning(mc_ctx *ctx, mc_tuning *t)
{
    if (!ctx || !t) return MC_EINVAL;
    *t = ctx->tune;
    t->lookup_ilp = lookup_ilp(ctx);
    t->tail_particles = (int32_t)tail_particles(ctx);
    if (!t->sort_min) t->sort_min = (int32_t)kDefaultSortMin;
    if (!t->collide_sort_min) t->collide_sort_min = t->sort_min;
    if (!t->loops) t->loops = 1;
    if (!t->in_flight) t->in_flight = (int32_t)kDefaultInFlight;
    if (!t->set_tile_histories) t->set_tile_histories = WG;
    if (!t->set_grid) t->set_grid = 2 * ctx->n_cu;
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

// The parts of the static scratch for a sorted lookup of up to n pairs,
// each 256-byte aligned; returns the bytes they span.
static size_t carve_noalloc(unsigned char *base, size_t n, uint32_t **perm, uint32_t **keys, SortBufs *sb)
{
    size_t off = 0;
    auto take = [&](size_t words) {
        uint32_t *p = reinterpret_cast<uint32_t *>(base + off);
        off += (words * sizeof(uint32_t) + 255) & ~size_t(255);
        return p;
    };
    *perm = take(n);
    *keys = take(n);
    sb->kA = take(n);
    sb->kB = take(n);
    sb->vA = take(n);
    sb->vB = take(n);
    const size_t tiles = sort_tile_count(n), chunks = sort_chunk_count(n);
    sb->tile_hist = take(tiles * 256);
    sb->chunk_total = take(chunks * 256);
    sb->chunk_off = take((chunks + 1) * 256);
    return off;
}

int mc_lookup_macro_noalloc(mc_ctx *ctx, size_t n, const double *E, const int32_t *mat, double *sig_a,
                            double *sig_s, int32_t sorted)
{
    if (!ctx) return MC_EINVAL;
    if (!ctx->have_mat) return fail(ctx, MC_ESTATE, "mc_lookup_macro_noalloc: no materials");
    if (n == 0) return MC_OK;
    if (n > MC_NOALLOC_MAX_LOOKUPS)
        return fail(ctx, MC_EINVAL, "mc_lookup_macro_noalloc: n = " + std::to_string(n) + " above the maximum of " +
                                        std::to_string(MC_NOALLOC_MAX_LOOKUPS) + " lookups per call");
    if (!E || !mat) return fail(ctx, MC_EINVAL, "mc_lookup_macro_noalloc: bad arguments");
    if (!ctx->noalloc_scratch) return fail(ctx, MC_ESTATE, "mc_lookup_macro_noalloc: no scratch on this device");
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
        uint32_t *perm = nullptr, *keys = nullptr;
        SortBufs sb;
        const size_t used = carve_noalloc(static_cast<unsigned char *>(ctx->noalloc_scratch), n, &perm, &keys, &sb);
        if (used > MC_NOALLOC_SCRATCH_BYTES)
            return fail(ctx, MC_EINVAL, "mc_lookup_macro_noalloc: scratch too small for n");
        // the radix counts add into chunk_total, which an earlier call (or an
        // interrupted one) may have left non-zero: clear this call's part
        HIPCHK(launch_fill_u32(sb.chunk_total, sort_chunk_count(n) * 256, 0u, ctx->stream));
        HIPCHK(launch_sort(ctx->xs, nullptr, nullptr, (uint32_t)n, E, mat, sb, ctx->n_keys, perm, keys,
                           ctx->stream));
        l.list = perm;
        l.keys = keys;
    }
    HIPCHK(launch_lookup(l, ctx->stream));
    return MC_OK;
}

int mc_lookup_channels(mc_ctx *ctx, size_t n, const double *E, const int32_t *mat, double *out, double *sig_a,
                       double *sig_s)
{
    if (!ctx) return MC_EINVAL;
    if (!ctx->have_mat) return fail(ctx, MC_ESTATE, "mc_lookup_channels: no materials");
    if (n == 0) return MC_OK;
    if (!ctx->n_chan) return fail(ctx, MC_ESTATE, "mc_lookup_channels: no reaction channels");
    if (n >= (1ull << 31) || !E || !mat || !out) return fail(ctx, MC_EINVAL, "mc_lookup_channels: bad arguments");
    HIPCHK(hipSetDevice(ctx->device));
    LookupLaunch l;
    l.xs = ctx->xs;
    l.n_bound = (uint32_t)n;
    l.E = E;
    l.mat = mat;
    l.Sa = sig_a;
    l.Ss = sig_s;
    l.ilp = lookup_ilp(ctx);
    l.sx = out;
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
    s.lookup_bytes += (36ull + 8ull * (uint64_t)ctx->n_chan) * n + (56ull + 16ull * (uint64_t)ctx->n_chan) * nuc;
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


// ---------------------------------------------------------------------------
// problem set
// ---------------------------------------------------------------------------
static void drop_graph(mc_ctx *ctx)
{
    if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    ctx->gexec = nullptr;
    ctx->graph = nullptr;
}

// Tiles of T histories, problems in cost order, and the rows they write.
static int build_set_tiles(mc_ctx *ctx, uint32_t T)
{
    HIPCHK(hipStreamSynchronize(ctx->stream));
    drop_graph(ctx);
    ctx->set_tile_bufs.release();
    std::vector<SetTile> tiles;
    std::vector<SetProblem> probs = ctx->set_probs;
    uint64_t row = 0;
    for (int32_t p : ctx->set_order) {
        SetProblem &P = probs[p];
        P.first_tile = (uint32_t)tiles.size();
        for (uint64_t h = 0; h < P.histories; h += T) {
            SetTile t;
            t.problem = p;
            t.first = (uint32_t)h;
            t.count = (uint32_t)std::min<uint64_t>(T, P.histories - h);
            t.row = row;
            row += (uint64_t)P.g.n_bins;
            tiles.push_back(t);
        }
        P.n_tiles = (uint32_t)tiles.size() - P.first_tile;
    }
    if (tiles.size() >= (1ull << 31)) return fail(ctx, MC_EINVAL, "problem set: too many tiles");
    Buffers &B = ctx->set_tile_bufs;
    SetProblem *d_probs;
    SetTile *d_tiles;
    int rc = upload(ctx, B, &d_probs, probs.data(), probs.size());
    if (!rc) rc = upload(ctx, B, &d_tiles, tiles.data(), tiles.size());
    if (!rc) rc = dalloc(ctx, B, &ctx->set.tl, (size_t)row);
    if (!rc) rc = dalloc(ctx, B, &ctx->set.coll, (size_t)row);
    if (!rc) rc = dalloc(ctx, B, &ctx->set.glob, tiles.size() * N_GLOBAL);
    if (rc) {
        B.release();
        ctx->set_tile_hist = 0;
        return rc;
    }
    ctx->set.problems = d_probs;
    ctx->set.tiles = d_tiles;
    ctx->set.n_tiles = (uint32_t)tiles.size();
    ctx->set.n_rows_doubles = (size_t)row;
    ctx->set_probs = probs;
    ctx->set_tile_hist = T;
    return MC_OK;
}

int mc_set_problem_set(mc_ctx *ctx, int32_t n_problems, const mc_problem_desc *pr, int32_t n_hash_bins)
{
    if (!ctx) return MC_EINVAL;
    if (n_problems < 1 || !pr || n_hash_bins < 1) return fail(ctx, MC_EINVAL, "mc_set_problem_set: bad arguments");
    HIPCHK(hipSetDevice(ctx->device));
    HostXs H;
    std::vector<int32_t> mat_base(n_problems);
    for (int32_t p = 0; p < n_problems; ++p) {
        const std::string who = "problem " + std::to_string(p) + ": ";
        if (!pr[p].geometry) return fail(ctx, MC_EINVAL, who + "no geometry");
        if (pr[p].histories < 1 || pr[p].histories >= (1ull << 31))
            return fail(ctx, MC_EINVAL, who + "histories must be in [1, 2^31)");
        mat_base[p] = (int32_t)H.mat_len.size();
        const NuclideInput in{pr[p].n_nuc, pr[p].grid_len, pr[p].E, pr[p].sig_c, pr[p].sig_s, pr[p].awr,
                              pr[p].n_mat, pr[p].mat_len, pr[p].mat_nuc, pr[p].mat_dens};
        int rc = append_xs(ctx, H, in, who);
        if (rc) return rc;
    }
    int rc = finish_xs(ctx, H, n_hash_bins);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    drop_graph(ctx);
    ctx->set_tile_bufs.release();
    ctx->set_bufs.release();
    ctx->have_set = false;
    ctx->set_tile_hist = 0;
    Buffers &B = ctx->set_bufs;
    rc = upload_xs(ctx, H, n_hash_bins, B, ctx->set_xs);
    std::vector<SetProblem> probs(n_problems);
    std::vector<double> cost(n_problems);
    uint64_t stat = 0, log_off = 0;
    int32_t max_bins = 1;
    for (int32_t p = 0; p < n_problems && !rc; ++p) {
        const std::string who = "problem " + std::to_string(p) + ": ";
        GeomDev g{};
        rc = build_geometry(ctx, pr[p].geometry, pr[p].n_mat, mat_base[p], B, g, who);
        if (rc) break;
        if (g.tally_kind == TALLY_MESH) {
            rc = fail(ctx, MC_EINVAL, who + "mesh tallies are not supported in a problem set");
            break;
        }
        SetProblem &P = probs[p];
        P = SetProblem{};
        P.g = g;
        P.seed = pr[p].seed;
        P.histories = pr[p].histories;
        P.pid_base = pr[p].first_pid;
        P.log_off = log_off;
        P.stat_off = stat;
        log_off += pr[p].histories;
        stat += 2ull * (uint64_t)g.n_bins + N_GLOBAL;
        max_bins = std::max(max_bins, g.n_bins);
        int32_t nk_max = 1;
        for (int32_t m = 0; m < pr[p].n_mat; ++m) nk_max = std::max(nk_max, pr[p].mat_len[m]);
        cost[p] = (double)pr[p].histories * (double)nk_max;
    }
    if (!rc) rc = dalloc(ctx, B, &ctx->set.S1, stat);
    if (!rc) rc = dalloc(ctx, B, &ctx->set.S2, stat);
    if (!rc) rc = dalloc(ctx, B, &ctx->set.next_tile, 1);
    if (!rc) rc = dalloc(ctx, B, &ctx->set.batch, 1);
    if (!rc) rc = dalloc(ctx, B, &ctx->set.lost, 1);
    if (rc) {
        B.release();
        return rc;
    }
    HIPCHK(launch_fill_f64(ctx->set.S1, stat, 0.0, ctx->stream));
    HIPCHK(launch_fill_f64(ctx->set.S2, stat, 0.0, ctx->stream));
    HIPCHK(launch_fill_u32(reinterpret_cast<uint32_t *>(ctx->set.batch), 2, 0u, ctx->stream));
    HIPCHK(launch_fill_u32(reinterpret_cast<uint32_t *>(ctx->set.lost), 2, 0u, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->set.n_problems = n_problems;
    ctx->set.log = nullptr;
    ctx->set_probs = probs;
    ctx->set_order.resize(n_problems);
    for (int32_t p = 0; p < n_problems; ++p) ctx->set_order[p] = p;
    // costliest problems first, so that the queue ends on small tiles
    std::stable_sort(ctx->set_order.begin(), ctx->set_order.end(),
                     [&](int32_t a, int32_t b) { return cost[a] > cost[b]; });
    ctx->set_max_bins = max_bins;
    {
        uint64_t h = fnv(fnv_vec(fnv_vec(1469598103934665603ull, H.glen), H.mnucid), &n_hash_bins, sizeof(n_hash_bins));
        for (const SetProblem &P : probs) h = fnv(geom_signature(h, P.g), &P.histories, sizeof(P.histories));
        ctx->set_sig = h;
    }
    ctx->set_batches = 0;
    ctx->set_histories = log_off;
    ctx->have_set = true;
    return MC_OK;
}

int mc_reset_problem_set(mc_ctx *ctx)
{
    if (!ctx) return MC_EINVAL;
    if (!ctx->have_set) return fail(ctx, MC_ESTATE, "no problem set");
    HIPCHK(hipSetDevice(ctx->device));
    size_t stat = 0;
    for (const SetProblem &P : ctx->set_probs) stat += 2ull * (size_t)P.g.n_bins + N_GLOBAL;
    HIPCHK(launch_fill_f64(ctx->set.S1, stat, 0.0, ctx->stream));
    HIPCHK(launch_fill_f64(ctx->set.S2, stat, 0.0, ctx->stream));
    HIPCHK(launch_fill_u32(reinterpret_cast<uint32_t *>(ctx->set.batch), 2, 0u, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->set_batches = 0;
    return MC_OK;
}

int mc_run_problem_set(mc_ctx *ctx, const mc_set_opts *opts_in)
{
    if (!ctx) return MC_EINVAL;
    if (!ctx->have_set) return fail(ctx, MC_ESTATE, "mc_run_problem_set: no problem set");
    HIPCHK(hipSetDevice(ctx->device));
    mc_set_opts opts{};
    if (opts_in) opts = *opts_in;
    const uint32_t T = ctx->tune.set_tile_histories > 0 ? (uint32_t)ctx->tune.set_tile_histories : (uint32_t)WG;
    if (T != ctx->set_tile_hist) {
        int rc = build_set_tiles(ctx, T);
        if (rc) return rc;
    }
    const uint32_t grid = ctx->tune.set_grid > 0 ? (uint32_t)ctx->tune.set_grid : (uint32_t)(2 * ctx->n_cu);
    const int64_t max_events = opts.max_events > 0 ? opts.max_events : kDefaultMaxEvents;
    HistLog *log = static_cast<HistLog *>(opts.history_log);
    hipStream_t st = ctx->stream;
    HIPCHK(launch_fill_u32(reinterpret_cast<uint32_t *>(ctx->set.lost), 2, 0u, st));
    HIPCHK(hipEventRecord(ctx->ev_batch0, st));
    if (opts.use_graph && !log) {
        if (!ctx->gexec || ctx->graph_grid != grid || ctx->graph_tile != T || ctx->graph_max_events != max_events) {
            drop_graph(ctx);
            if (!ctx->cap_stream) HIPCHK(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
            HIPCHK(hipStreamSynchronize(st));
            HIPCHK(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
            const hipError_t le = launch_problem_set(ctx->set, ctx->set_xs, max_events, grid, ctx->set_max_bins,
                                                     ctx->cap_stream);
            hipGraph_t gr = nullptr;
            const hipError_t ce = hipStreamEndCapture(ctx->cap_stream, &gr);
            if (le != hipSuccess || ce != hipSuccess) {
                if (gr) (void)hipGraphDestroy(gr);
                return fail(ctx, MC_EHIP, std::string("graph capture: ") + hipGetErrorString(le != hipSuccess ? le : ce));
            }
            ctx->graph = gr;
            HIPCHK(hipGraphInstantiate(&ctx->gexec, ctx->graph, nullptr, nullptr, 0));
            ctx->graph_grid = grid;
            ctx->graph_tile = T;
            ctx->graph_max_events = max_events;
        }
        HIPCHK(hipGraphLaunch(ctx->gexec, st));
    } else {
        SetDev s = ctx->set;
        s.log = log;
        HIPCHK(launch_problem_set(s, ctx->set_xs, max_events, grid, ctx->set_max_bins, st));
    }
    HIPCHK(hipEventRecord(ctx->ev_batch1, st));
    unsigned long long lost = 0;
    HIPCHK(hipMemcpyAsync(&lost, ctx->set.lost, sizeof(lost), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, ctx->ev_batch0, ctx->ev_batch1));
    mc_stats s{};
    s.batch_ms = ms;
    s.lost = lost;
    ctx->stats = s;
    ctx->set_batches += 1;
    if (lost > 0) return fail(ctx, MC_ELOST, std::to_string(lost) + " particles lost (event cap reached)");
    return MC_OK;
}

int mc_get_problem_tallies(mc_ctx *ctx, int32_t problem, int32_t tally_id, double *mean, double *stderr_,
                           size_t n_bins, mc_tally_meta *meta)
{
    if (!ctx) return MC_EINVAL;
    if (!ctx->have_set) return fail(ctx, MC_ESTATE, "no problem set");
    if (problem < 0 || problem >= ctx->set.n_problems) return fail(ctx, MC_EINVAL, "problem out of range");
    if (tally_id < 0 || tally_id > 2) return fail(ctx, MC_EINVAL, "unknown tally id");
    const SetProblem &P = ctx->set_probs[problem];
    const size_t nbp = (size_t)P.g.n_bins;
    const size_t nb = tally_id == MC_T_GLOBAL ? (size_t)N_GLOBAL : nbp;
    if (n_bins != nb) return fail(ctx, MC_EINVAL, "n_bins does not match the tally (" + std::to_string(nb) + ")");
    const size_t off = P.stat_off + (size_t)tally_id * nbp;
    HIPCHK(hipSetDevice(ctx->device));
    std::vector<double> s1(nb), s2(nb);
    HIPCHK(hipMemcpyAsync(s1.data(), ctx->set.S1 + off, nb * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipMemcpyAsync(s2.data(), ctx->set.S2 + off, nb * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    const double B = (double)ctx->set_batches;
    for (size_t k = 0; k < nb; ++k) {
        const double m = B > 0 ? s1[k] / B : 0.0;
        if (mean) mean[k] = m;
        if (stderr_) stderr_[k] = (B > 1) ? std::sqrt(std::max(s2[k] / B - m * m, 0.0) / (B - 1.0)) : 0.0;
    }
    if (meta) {
        meta->n_batches = ctx->set_batches;
        meta->n_bins = nb;
        meta->histories = ctx->set_batches * P.histories;
    }
    return MC_OK;
}


// ---------------------------------------------------------------------------
// autotuner
// ---------------------------------------------------------------------------
static std::string sig_text(const mc_ctx *ctx, const char *what, uint64_t sig)
{
    char buf[128];
    std::snprintf(buf, sizeof buf, "%s-%s-%016llx", what, ctx->arch.c_str(), (unsigned long long)sig);
    std::string s(buf);
    for (char &c : s)
        if (c == ' ' || c == ':') c = '_';
    return s;
}

static bool cache_lookup(const char *path, const std::string &sig, mc_tuning &t)
{
    if (!path) return false;
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        char s[200];
        mc_tuning r{};
        double ms = 0.0;
        // fields: signature, lookup_ilp, tail, sort_min, in_flight, set tile,
        // set grid, best ms, collide_sort_min, loops (the last two absent in
        // older lines: 0)
        const int got = std::sscanf(line, "%199s %d %d %d %d %d %d %lf %d %d", s, &r.lookup_ilp, &r.tail_particles,
                                    &r.sort_min, &r.in_flight, &r.set_tile_histories, &r.set_grid, &ms,
                                    &r.collide_sort_min, &r.loops);
        if (got >= 8 && sig == s) {
            t = r;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

static void cache_store(const char *path, const std::string &sig, const mc_tuning &t, double ms)
{
    if (!path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s %d %d %d %d %d %d %.4f %d %d\n", sig.c_str(), t.lookup_ilp, t.tail_particles, t.sort_min,
                 t.in_flight, t.set_tile_histories, t.set_grid, ms, t.collide_sort_min, t.loops);
    std::fclose(f);
}

int mc_autotune(mc_ctx *ctx, uint64_t seed, uint64_t first_pid, uint64_t n, const char *cache_path, mc_tuning *best)
{
    if (!ctx || n == 0) return MC_EINVAL;
    if (!ctx->have_geom) return fail(ctx, MC_ESTATE, "mc_autotune: materials and geometry first");
    uint64_t key = fnv(ctx->geom_sig, &n, sizeof(n));
    if (ctx->n_chan) key = fnv(key, &ctx->n_chan, sizeof(ctx->n_chan));  // channels change the lookup kernel
    const std::string sig = sig_text(ctx, "single", key);
    mc_tuning t = ctx->tune;
    if (cache_lookup(cache_path, sig, t)) {
        ctx->tune = t;
        if (best) *best = t;
        return MC_OK;
    }
    mc_tuning cur{};
    int rc = mc_get_tuning(ctx, &cur);
    if (rc) return rc;
    const int32_t n_cap = (int32_t)std::min<uint64_t>(n, kMaxTunedInFlight);
    cur.in_flight = (int32_t)std::min<uint64_t>(n, kDefaultInFlight);
    cur.collide_sort_min = 0;  // follows sort_min unless the search turns it off
    // each trial, timed per batch through mc_run_batches (consecutive batches,
    // each event loop taking whole batches): 12 batches (whole rounds for 1
    // to 4 loops, so that loops > 1 shows its overlap of consecutive
    // batches); batches of 2^22 histories or more: one round, one batch per
    // loop (at least two)
    const bool large = n >= (1ull << 22);
    auto trial = [&](const mc_tuning &c, double &ms) -> int {
        ctx->tune = c;
        const uint64_t nb = large ? (uint64_t)std::max(2, (int)c.loops) : 12u;
        const int r = mc_run_batches(ctx, seed, first_pid, n, nb, nullptr);
        ms = ctx->stats.batch_ms / (double)nb;
        return r;
    };
    double best_ms = 0.0;
    rc = trial(cur, best_ms);  // warm-up (code and bank), then the baseline
    if (!rc) rc = trial(cur, best_ms);
    // coordinate descent, two sweeps over the axes (tail and sort interact)
    const int32_t ilps[] = {1, 2, 4};
    const int32_t tails[] = {8192, 32768, 131072, 262144};
    const int32_t sorts[] = {4096, 16384, 65536, 262144, (int32_t)kSortNever};
    // per loop: a quarter, a third or half of the batch (so 4, 3 or 2 loops
    // hold it all in flight at once), fixed sizes, the whole batch
    const int32_t flights[] = {std::max(1024, n_cap / 4), std::max(1024, n_cap / 3), std::max(1024, n_cap / 2),
                               1 << 20, 1 << 22, n_cap};
    const int32_t csorts[] = {0, (int32_t)kSortNever};
    const int32_t loops[] = {1, 2, 3, 4};
    // the loop count first: whether a sort pays depends on what overlaps it
    const int32_t *axes[] = {loops, tails, sorts, ilps, flights, csorts};
    const int counts[] = {4, 4, 5, 3, 6, 2};
    for (int sweep = 0; sweep < 2 && !rc; ++sweep) {
        for (int axis = 0; axis < 6 && !rc; ++axis) {
            for (int k = 0; k < counts[axis] && !rc; ++k) {
                mc_tuning c = cur;
                const int32_t v = axes[axis][k];
                if (axis == 0) c.loops = v;
                if (axis == 1) c.tail_particles = v;
                if (axis == 2) c.sort_min = v;
                if (axis == 3) c.lookup_ilp = v;
                if (axis == 4) c.in_flight = std::min(v, n_cap);
                if (axis == 5) c.collide_sort_min = v;
                if (std::memcmp(&c, &cur, sizeof c) == 0) continue;
                double ms = 0.0;
                rc = trial(c, ms);
                if (!rc && ms < best_ms) {
                    best_ms = ms;
                    cur = c;
                }
            }
        }
    }
    ctx->tune = cur;
    if (rc) return rc;
    rc = reset_tallies(ctx);
    if (rc) return rc;
    cache_store(cache_path, sig, cur, best_ms);
    if (best) *best = cur;
    return MC_OK;
}

int mc_autotune_problem_set(mc_ctx *ctx, const char *cache_path, mc_tuning *best)
{
    if (!ctx) return MC_EINVAL;
    if (!ctx->have_set) return fail(ctx, MC_ESTATE, "mc_autotune_problem_set: no problem set");
    const std::string sig = sig_text(ctx, "set", ctx->set_sig);
    mc_tuning t = ctx->tune;
    if (cache_lookup(cache_path, sig, t)) {
        ctx->tune = t;
        if (best) *best = t;
        return MC_OK;
    }
    mc_tuning cur{};
    int rc = mc_get_tuning(ctx, &cur);
    if (rc) return rc;
    auto trial = [&](const mc_tuning &c, double &ms) -> int {
        ctx->tune = c;
        const int r = mc_run_problem_set(ctx, nullptr);
        ms = ctx->stats.batch_ms;
        return r;
    };
    double best_ms = 0.0;
    rc = trial(cur, best_ms);  // warm-up
    if (!rc) rc = trial(cur, best_ms);
    const int32_t tiles[] = {256, 512, 1024, 2048};
    const int32_t per_cu[] = {1, 2, 4, 8};
    mc_tuning pick = cur;
    for (int a = 0; a < 4 && !rc; ++a) {
        for (int b = 0; b < 4 && !rc; ++b) {
            mc_tuning c = cur;
            c.set_tile_histories = tiles[a];
            c.set_grid = per_cu[b] * ctx->n_cu;
            double ms = 0.0;
            rc = trial(c, ms);
            if (!rc && ms < best_ms) {
                best_ms = ms;
                pick = c;
            }
        }
    }
    cur = pick;
    ctx->tune = cur;
    if (rc) return rc;
    rc = mc_reset_problem_set(ctx);
    if (rc) return rc;
    cache_store(cache_path, sig, cur, best_ms);
    if (best) *best = cur;
    return MC_OK;
}


// ---------------------------------------------------------------------------
// importance network
// ---------------------------------------------------------------------------
static int mlp_alloc(mc_ctx *ctx)
{
    if (ctx->have_mlp) return MC_OK;
    Buffers &B = ctx->mlp_bufs;
    int rc = dalloc(ctx, B, &ctx->theta, MLP_NPAR);
    if (!rc) rc = dalloc(ctx, B, &ctx->mom, MLP_NPAR);
    if (!rc) rc = dalloc(ctx, B, &ctx->vel, MLP_NPAR);
    if (!rc) rc = dalloc(ctx, B, &ctx->grad, MLP_NPAR + 1);
    if (!rc) rc = dalloc(ctx, B, &ctx->inv_wsum, 1);
    if (!rc) rc = dalloc(ctx, B, &ctx->W1b, 256);
    if (!rc) rc = dalloc(ctx, B, &ctx->W2b, 4096);
    if (!rc) rc = dalloc(ctx, B, &ctx->W2tb, 4096);
    if (!rc) rc = dalloc(ctx, B, &ctx->w3b, 64);
    if (rc) B.release();
    return rc;
}

// Adam state to zero and the BF16 copies from the FP32 parameters.
static int mlp_reset_state(mc_ctx *ctx)
{
    HIPCHK(launch_fill_u32(reinterpret_cast<uint32_t *>(ctx->mom), MLP_NPAR, 0u, ctx->stream));
    HIPCHK(launch_fill_u32(reinterpret_cast<uint32_t *>(ctx->vel), MLP_NPAR, 0u, ctx->stream));
    HIPCHK(launch_mlp_sync(ctx->theta, ctx->W1b, ctx->W2b, ctx->W2tb, ctx->w3b, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->mlp_step = 0;
    ctx->have_mlp = true;
    return MC_OK;
}

int mc_mlp_set(mc_ctx *ctx, const float *params)
{
    if (!ctx || !params) return MC_EINVAL;
    for (int j = 0; j < MLP_NPAR; ++j)
        if (!std::isfinite(params[j])) return fail(ctx, MC_EINVAL, "mc_mlp_set: parameter " + std::to_string(j) + " not finite");
    HIPCHK(hipSetDevice(ctx->device));
    int rc = mlp_alloc(ctx);
    if (rc) return rc;
    HIPCHK(hipMemcpyAsync(ctx->theta, params, MLP_NPAR * sizeof(float), hipMemcpyHostToDevice, ctx->stream));
    return mlp_reset_state(ctx);
}

int mc_mlp_get(mc_ctx *ctx, float *params)
{
    if (!ctx || !params) return MC_EINVAL;
    if (!ctx->have_mlp) return fail(ctx, MC_ESTATE, "mc_mlp_get: no network (mc_mlp_set first)");
    HIPCHK(hipSetDevice(ctx->device));
    HIPCHK(hipMemcpyAsync(params, ctx->theta, MLP_NPAR * sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return MC_OK;
}

int mc_mlp_forward(mc_ctx *ctx, size_t n, const float *features, float *out)
{
    if (!ctx) return MC_EINVAL;
    if (!ctx->have_mlp) return fail(ctx, MC_ESTATE, "mc_mlp_forward: no network (mc_mlp_set first)");
    if (n == 0) return MC_OK;
    if (!features || !out || n >= (1ull << 31)) return fail(ctx, MC_EINVAL, "mc_mlp_forward: bad arguments");
    HIPCHK(hipSetDevice(ctx->device));
    HIPCHK(launch_mlp_forward(mlp_dev(ctx), (uint32_t)n, features, out, ctx->stream));
    return MC_OK;
}

static int mlp_scratch(mc_ctx *ctx, size_t n, int32_t steps)
{
    const size_t need = mlp_partial_floats((uint32_t)n);
    if (need <= ctx->mlp_scratch_n && steps <= ctx->mlp_loss_cap) return MC_OK;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->mlp_scratch_bufs.release();
    ctx->mlp_scratch_n = 0;
    ctx->mlp_loss_cap = 0;
    const size_t n2 = std::max(need, ctx->mlp_scratch_n);
    const int32_t s2 = std::max<int32_t>(steps, 1);
    int rc = dalloc(ctx, ctx->mlp_scratch_bufs, &ctx->mlp_partial, n2);
    if (!rc) rc = dalloc(ctx, ctx->mlp_scratch_bufs, &ctx->mlp_loss, (size_t)s2);
    if (rc) {
        ctx->mlp_scratch_bufs.release();
        return rc;
    }
    ctx->mlp_scratch_n = n2;
    ctx->mlp_loss_cap = s2;
    return MC_OK;
}

int mc_mlp_grad(mc_ctx *ctx, size_t n, const float *features, const float *target, const float *weight,
                float *grad, float *loss)
{
    if (!ctx) return MC_EINVAL;
    if (!ctx->have_mlp) return fail(ctx, MC_ESTATE, "mc_mlp_grad: no network (mc_mlp_set first)");
    if (n == 0 || n >= (1ull << 24) || !features || !target || !weight)
        return fail(ctx, MC_EINVAL, "mc_mlp_grad: bad arguments");
    HIPCHK(hipSetDevice(ctx->device));
    int rc = mlp_scratch(ctx, n, 1);
    if (rc) return rc;
    HIPCHK(launch_mlp_wsum(weight, (uint32_t)n, ctx->inv_wsum, ctx->stream));
    HIPCHK(launch_mlp_grad(mlp_dev(ctx), (uint32_t)n, features, target, weight, ctx->inv_wsum, ctx->mlp_partial,
                           ctx->grad, ctx->stream));
    std::vector<float> g(MLP_NPAR + 1);
    HIPCHK(hipMemcpyAsync(g.data(), ctx->grad, g.size() * sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (grad) std::memcpy(grad, g.data(), MLP_NPAR * sizeof(float));
    if (loss) *loss = g[MLP_NPAR];
    return MC_OK;
}

static int mlp_train_loop(mc_ctx *ctx, size_t n, const float *features, const float *target, const float *weight,
                          int32_t steps, float lr, float *loss_curve)
{
    int rc = mlp_scratch(ctx, n, steps);
    if (rc) return rc;
    hipStream_t st = ctx->stream;
    HIPCHK(launch_mlp_wsum(weight, (uint32_t)n, ctx->inv_wsum, st));
    for (int32_t k = 0; k < steps; ++k) {
        HIPCHK(launch_mlp_grad(mlp_dev(ctx), (uint32_t)n, features, target, weight, ctx->inv_wsum, ctx->mlp_partial,
                               ctx->grad, st));
        HIPCHK(hipMemcpyAsync(ctx->mlp_loss + k, ctx->grad + MLP_NPAR, sizeof(float), hipMemcpyDeviceToDevice, st));
        ctx->mlp_step += 1;
        HIPCHK(launch_mlp_adam(ctx->theta, ctx->mom, ctx->vel, ctx->grad, ctx->mlp_step, lr, ctx->W1b, ctx->W2b,
                               ctx->W2tb, ctx->w3b, st));
    }
    if (loss_curve)
        HIPCHK(hipMemcpyAsync(loss_curve, ctx->mlp_loss, (size_t)steps * sizeof(float), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return MC_OK;
}

int mc_mlp_train(mc_ctx *ctx, size_t n, const float *features, const float *target, const float *weight,
                 int32_t steps, float lr, float *loss_curve)
{
    if (!ctx) return MC_EINVAL;
    if (!ctx->have_mlp) return fail(ctx, MC_ESTATE, "mc_mlp_train: no network (mc_mlp_set first)");
    if (n == 0 || n >= (1ull << 24) || !features || !target || !weight || steps < 1 || !(lr > 0.0f))
        return fail(ctx, MC_EINVAL, "mc_mlp_train: bad arguments");
    HIPCHK(hipSetDevice(ctx->device));
    return mlp_train_loop(ctx, n, features, target, weight, steps, lr, loss_curve);
}

int mc_mlp_init(mc_ctx *ctx, uint64_t seed)
{
    if (!ctx) return MC_EINVAL;
    HIPCHK(hipSetDevice(ctx->device));
    int rc = mlp_alloc(ctx);
    if (rc) return rc;
    HIPCHK(launch_mlp_init(ctx->theta, seed, ctx->stream));
    return mlp_reset_state(ctx);
}

static int imp_sample_args(mc_ctx *ctx, const mc_train_opts *o, int32_t nx, int32_t ne, double x0, double x1,
                           ImpSampleArgs &a, const std::string &who)
{
    if (!o) return fail(ctx, MC_EINVAL, who + ": options required");
    if (o->replicas < 1 || o->replicas > 64) return fail(ctx, MC_EINVAL, who + ": replicas outside [1, 64]");
    if (!(o->min_credits >= 1.0) || !(o->rel_floor >= 0.0) || !(o->length > 0.0))
        return fail(ctx, MC_EINVAL, who + ": need min_credits >= 1, rel_floor >= 0, length > 0");
    if (nx < 1 || ne < 1 || (int64_t)nx * ne > (1 << 20) || !(x1 > x0))
        return fail(ctx, MC_EINVAL, who + ": bad importance grid");
    a.nx = nx;
    a.ne = ne;
    a.x0 = x0;
    a.x1 = x1;
    a.length = o->length;
    a.replicas = o->replicas;
    a.min_credits = o->min_credits;
    a.rel_floor = o->rel_floor;
    a.seed = o->seed;
    return MC_OK;
}

int mc_importance_samples(mc_ctx *ctx, const double *num, const double *den, const double *cnt, int32_t nx,
                          int32_t ne, double x0, double x1, const mc_train_opts *opts, float *features,
                          float *target, float *weight, int32_t *n_samples)
{
    if (!ctx) return MC_EINVAL;
    ImpSampleArgs a{};
    int rc = imp_sample_args(ctx, opts, nx, ne, x0, x1, a, "mc_importance_samples");
    if (rc) return rc;
    if (!num || !den || !cnt || !features || !target || !weight || !n_samples)
        return fail(ctx, MC_EINVAL, "mc_importance_samples: NULL argument");
    HIPCHK(hipSetDevice(ctx->device));
    const size_t cells = (size_t)nx * (size_t)ne;
    Buffers tmp;
    double *d_num = nullptr, *d_den = nullptr, *d_cnt = nullptr;
    int32_t *d_n = nullptr;
    rc = upload(ctx, tmp, &d_num, num, cells);
    if (!rc) rc = upload(ctx, tmp, &d_den, den, cells);
    if (!rc) rc = upload(ctx, tmp, &d_cnt, cnt, cells);
    if (!rc) rc = dalloc(ctx, tmp, &d_n, 1);
    if (rc) {
        tmp.release();
        return rc;
    }
    a.num = d_num;
    a.den = d_den;
    a.cnt = d_cnt;
    a.X = features;
    a.T = target;
    a.W = weight;
    a.n_out = d_n;
    a.range_out = nullptr;
    hipError_t e = launch_imp_samples(a, ctx->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(n_samples, d_n, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    tmp.release();
    if (e != hipSuccess) return fail(ctx, MC_EHIP, std::string("mc_importance_samples: ") + hipGetErrorString(e));
    return MC_OK;
}

int mc_importance_train(mc_ctx *ctx, const mc_train_opts *opts, float *loss_curve, int32_t *n_samples,
                        float *target_range)
{
    if (!ctx) return MC_EINVAL;
    if (!ctx->have_mlp) return fail(ctx, MC_ESTATE, "mc_importance_train: no network (mc_mlp_init or mc_mlp_set)");
    const mc_ww_desc &d = ctx->ww_desc;
    if (d.imp_nx < 1 || !ctx->imp_num) return fail(ctx, MC_ESTATE, "mc_importance_train: no importance grid");
    ImpSampleArgs a{};
    int rc = imp_sample_args(ctx, opts, d.imp_nx, d.imp_ne, d.imp_x0, d.imp_x1, a, "mc_importance_train");
    if (rc) return rc;
    if (opts->steps < 1 || !(opts->lr > 0.0f)) return fail(ctx, MC_EINVAL, "mc_importance_train: steps >= 1, lr > 0");
    HIPCHK(hipSetDevice(ctx->device));
    const size_t cap = (size_t)d.imp_nx * (size_t)d.imp_ne * (size_t)opts->replicas;
    if (cap > ctx->imp_sample_cap) {
        HIPCHK(hipStreamSynchronize(ctx->stream));
        ctx->imp_sample_bufs.release();
        ctx->imp_sample_cap = 0;
        Buffers &B = ctx->imp_sample_bufs;
        rc = dalloc(ctx, B, &ctx->imp_X, cap * 4);
        if (!rc) rc = dalloc(ctx, B, &ctx->imp_T, cap);
        if (!rc) rc = dalloc(ctx, B, &ctx->imp_W, cap);
        if (!rc) rc = dalloc(ctx, B, &ctx->imp_n, 1);
        if (!rc) rc = dalloc(ctx, B, &ctx->imp_range, 2);
        if (rc) {
            B.release();
            return rc;
        }
        ctx->imp_sample_cap = cap;
    }
    a.num = ctx->imp_num;
    a.den = ctx->imp_den;
    a.cnt = ctx->imp_cnt;
    a.X = ctx->imp_X;
    a.T = ctx->imp_T;
    a.W = ctx->imp_W;
    a.n_out = ctx->imp_n;
    a.range_out = ctx->imp_range;
    HIPCHK(launch_imp_samples(a, ctx->stream));
    int32_t n = 0;
    float range[2] = {0.f, 0.f};
    HIPCHK(hipMemcpyAsync(&n, ctx->imp_n, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipMemcpyAsync(range, ctx->imp_range, sizeof(range), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (n_samples) *n_samples = n;
    if (target_range && n > 0) {
        target_range[0] = range[0];
        target_range[1] = range[1];
    }
    if (n == 0) return fail(ctx, MC_ESTATE, "mc_importance_train: no cell has min_credits detector credits");
    return mlp_train_loop(ctx, (size_t)n, ctx->imp_X, ctx->imp_T, ctx->imp_W, opts->steps, opts->lr, loss_curve);
}

// ---------------------------------------------------------------------------
// weight windows and the forward importance estimate
// ---------------------------------------------------------------------------
int mc_set_weight_windows(mc_ctx *ctx, const mc_ww_desc *desc)
{
    if (!ctx) return MC_EINVAL;
    mc_ww_desc d{};
    if (desc) d = *desc;
    auto bad = [&](const std::string &m) { return fail(ctx, MC_EINVAL, "mc_set_weight_windows: " + m); };
    if (d.kind != MC_WW_OFF && d.kind != MC_WW_LINEAR && d.kind != MC_WW_MLP) return bad("unknown kind");
    if (d.kind != MC_WW_OFF) {
        if (d.n_max < 2 || d.n_max > 1000) return bad("n_max outside [2, 1000]");
        if (d.depth < 1 || d.depth > WW_MAX_DEPTH) return bad("depth outside [1, 64]");
        if (!(d.length > 0.0) || !(d.kappa > 0.0) || !(d.ratio > 1.0)) return bad("need length > 0, kappa > 0, ratio > 1");
        for (int k = 0; k < 3; ++k)
            if (!std::isfinite(d.lin[k])) return bad("lin not finite");
        if (!std::isfinite(d.ln_lo) || !std::isfinite(d.ln_hi)) return bad("ln_lo / ln_hi not finite");
    }
    if (d.imp_nx < 0 || d.imp_nx > IMP_MAX_NX) return bad("imp_nx outside [0, 256]");
    if (d.imp_nx > 0 && (d.imp_ne < 1 || d.imp_ne > IMP_MAX_NE || !(d.imp_x1 > d.imp_x0)))
        return bad("importance grid needs 1 <= imp_ne <= 64 and imp_x1 > imp_x0");
    if (d.imp_nx == 0) d.imp_ne = 0;
    HIPCHK(hipSetDevice(ctx->device));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    const bool same_shape = d.kind == ctx->ww_desc.kind && d.depth == ctx->ww_desc.depth &&
                            d.imp_nx == ctx->ww_desc.imp_nx && d.imp_ne == ctx->ww_desc.imp_ne;
    if (!same_shape) {
        ctx->ww_bufs.release();
        ctx->ww_cap = 0;
        ctx->ln_src = nullptr;
        ctx->ww = WwDev{};
    }
    const size_t cells = (size_t)d.imp_nx * (size_t)d.imp_ne;
    if (cells != (size_t)ctx->ww_desc.imp_nx * (size_t)ctx->ww_desc.imp_ne || (cells && !ctx->imp_num)) {
        ctx->imp_bufs.release();
        ctx->imp_num = ctx->imp_den = ctx->imp_cnt = nullptr;
        if (cells) {
            int rc = dalloc(ctx, ctx->imp_bufs, &ctx->imp_num, cells);
            if (!rc) rc = dalloc(ctx, ctx->imp_bufs, &ctx->imp_den, cells);
            if (!rc) rc = dalloc(ctx, ctx->imp_bufs, &ctx->imp_cnt, cells);
            if (rc) {
                ctx->imp_bufs.release();
                ctx->imp_num = ctx->imp_den = ctx->imp_cnt = nullptr;
                ctx->ww_desc = mc_ww_desc{};
                return rc;
            }
        }
    }
    ctx->ww_desc = d;
    if (cells) {
        HIPCHK(launch_fill_f64(ctx->imp_num, cells, 0.0, ctx->stream));
        HIPCHK(launch_fill_f64(ctx->imp_den, cells, 0.0, ctx->stream));
        HIPCHK(launch_fill_f64(ctx->imp_cnt, cells, 0.0, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
    }
    return MC_OK;
}

int mc_get_importance(mc_ctx *ctx, double *num, double *den, double *cnt, size_t n_cells)
{
    if (!ctx) return MC_EINVAL;
    const size_t cells = (size_t)ctx->ww_desc.imp_nx * (size_t)ctx->ww_desc.imp_ne;
    if (!cells) return fail(ctx, MC_ESTATE, "mc_get_importance: no importance grid (mc_set_weight_windows)");
    if (n_cells != cells) return fail(ctx, MC_EINVAL, "mc_get_importance: n_cells must be imp_nx * imp_ne");
    HIPCHK(hipSetDevice(ctx->device));
    if (num) HIPCHK(hipMemcpyAsync(num, ctx->imp_num, cells * 8, hipMemcpyDeviceToHost, ctx->stream));
    if (den) HIPCHK(hipMemcpyAsync(den, ctx->imp_den, cells * 8, hipMemcpyDeviceToHost, ctx->stream));
    if (cnt) HIPCHK(hipMemcpyAsync(cnt, ctx->imp_cnt, cells * 8, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return MC_OK;
}

}  // extern "C"
