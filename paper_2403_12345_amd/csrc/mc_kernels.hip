// mc_kernels.hip -- gfx950 kernels of the event-based transport loop.
//
// One iteration of the loop (paper section 2, "Event-Based Parallelism"):
//   queue    : rebuild the alive and lookup queues from the slot flags, refill
//              free slots with new source particles (section 2, "In-Flight
//              Particles")
//   sort     : order the lookup queue by (material, hash bin of E) (section 2,
//              "Sorting")
//   lookup   : macroscopic cross sections of every queued particle (the
//              dominant cost, section 2 "Sorting" and section 4.1)
//   advance  : distance to collision and to the nearest surface, move, score
//              track-length tallies (section 2 "Tallying")
//   split    : partition the alive queue into collide and cross queues
//   cross    : surface crossing (lattice step, cylinder, reflection, leakage)
//   collide  : capture or elastic scattering
// Every kernel uses 256-thread workgroups (4 wave64s).  Queue building and
// partitioning are stable and scan-based, so queue contents and tally sums are
// the same run to run.
#include "mc_device.h"
#include "mc_internal.h"

#pragma clang fp contract(off)

namespace mc {

// ---------------------------------------------------------------------------
// utilities
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(WG) k_fill_u8(uint8_t *p, size_t n, uint8_t v)
{
    for (size_t i = blockIdx.x * (size_t)WG + threadIdx.x; i < n; i += (size_t)gridDim.x * WG) p[i] = v;
}
__global__ void __launch_bounds__(WG) k_fill_u32(uint32_t *p, size_t n, uint32_t v)
{
    for (size_t i = blockIdx.x * (size_t)WG + threadIdx.x; i < n; i += (size_t)gridDim.x * WG) p[i] = v;
}
__global__ void __launch_bounds__(WG) k_fill_f64(double *p, size_t n, double v)
{
    for (size_t i = blockIdx.x * (size_t)WG + threadIdx.x; i < n; i += (size_t)gridDim.x * WG) p[i] = v;
}

// Block-wide ranks of up to three predicates over one round of 256 items:
// rank = items of the same predicate before this one (wave ballot, then the
// waves in order); total = items in the round.
struct Rank3 {
    uint32_t rank[3], total[3];
};

__device__ __forceinline__ Rank3 block_rank3(bool p0, bool p1, bool p2, uint32_t *lds)
{
    const int wave = threadIdx.x >> 6;
    const uint64_t lt = lanemask_lt();
    const uint64_t b0 = __ballot(p0), b1 = __ballot(p1), b2 = __ballot(p2);
    if (lane_id() == 0) {
        lds[0 * WAVES + wave] = __popcll(b0);
        lds[1 * WAVES + wave] = __popcll(b1);
        lds[2 * WAVES + wave] = __popcll(b2);
    }
    __syncthreads();
    Rank3 r;
    const uint64_t bb[3] = {b0, b1, b2};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        uint32_t pre = 0, tot = 0;
#pragma unroll
        for (int w = 0; w < WAVES; ++w) {
            const uint32_t c = lds[q * WAVES + w];
            pre += (w < wave) ? c : 0u;
            tot += c;
        }
        r.rank[q] = pre + (uint32_t)__popcll(bb[q] & lt);
        r.total[q] = tot;
    }
    __syncthreads();
    return r;
}

// Sum over the workgroup of three counts (any order: integers).
__device__ __forceinline__ void block_count3(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t *lds,
                                             uint32_t *out)
{
    c0 = wave_sum_u32(c0); c1 = wave_sum_u32(c1); c2 = wave_sum_u32(c2);
    const int wave = threadIdx.x >> 6;
    if (lane_id() == 0) { lds[wave] = c0; lds[WAVES + wave] = c1; lds[2 * WAVES + wave] = c2; }
    __syncthreads();
    if (threadIdx.x < 3) {
        uint32_t s = 0;
        for (int w = 0; w < WAVES; ++w) s += lds[threadIdx.x * WAVES + w];
        out[threadIdx.x] = s;
    }
}

// Exclusive prefix over tiles < t and the total over all tiles of three
// per-tile counts (each workgroup re-reads the few hundred tile counts).
__device__ __forceinline__ void tile_prefix3(const uint32_t *cnt, uint32_t n_tiles, uint32_t t,
                                             uint32_t *lds, uint32_t pre[3], uint32_t tot[3])
{
    uint32_t p[3] = {0, 0, 0}, s[3] = {0, 0, 0};
    for (uint32_t k = threadIdx.x; k < n_tiles; k += WG) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const uint32_t c = cnt[k * 3 + q];
            s[q] += c;
            p[q] += (k < t) ? c : 0u;
        }
    }
    uint32_t outp[3], outs[3];
    block_count3(p[0], p[1], p[2], lds, outp);
    __syncthreads();
    // broadcast via lds
    if (threadIdx.x < 3) lds[16 + threadIdx.x] = outp[threadIdx.x];
    __syncthreads();
    block_count3(s[0], s[1], s[2], lds, outs);
    __syncthreads();
    if (threadIdx.x < 3) lds[20 + threadIdx.x] = outs[threadIdx.x];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 3; ++q) { pre[q] = lds[16 + q]; tot[q] = lds[20 + q]; }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// queue building over the slots (one tile of 4096 slots per workgroup)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(WG) k_slots_count(BankDev bank)
{
    __shared__ uint32_t lds[32];
    const uint32_t base = blockIdx.x * (uint32_t)TILE;
    uint32_t ca = 0, cl = 0, cf = 0;
    for (int r = 0; r < TILE_ITEMS; ++r) {
        const uint32_t s = base + r * WG + threadIdx.x;
        if (s < bank.C) {
            const uint8_t f = bank.flags[s];
            ca += (f & F_ALIVE) ? 1u : 0u;
            cl += (f & F_LOOKUP) ? 1u : 0u;
            cf += (f & F_ALIVE) ? 0u : 1u;
        }
    }
    block_count3(ca, cl, cf, lds, bank.tile_cnt + blockIdx.x * 3);
}

// Sample a source particle into slot s (draw order: position for a box
// source, then the isotropic direction: cosine, azimuth).
__device__ __forceinline__ void init_particle(const BankDev &b, const GeomDev &g, uint32_t s,
                                              uint64_t pid, uint64_t seed)
{
    Rng rng(seed, pid, 0u, 0u);
    double x = g.src_pos[0], y = g.src_pos[1], z = g.src_pos[2];
    double u = g.src_dir[0], v = g.src_dir[1], w = g.src_dir[2];
    if (g.src_kind != SRC_BEAM) {
        if (g.src_kind == SRC_BOX) {
            x = g.src_box[0] + (g.src_box[1] - g.src_box[0]) * rng.next();
            y = g.src_box[2] + (g.src_box[3] - g.src_box[2]) * rng.next();
            z = g.src_box[4] + (g.src_box[5] - g.src_box[4]) * rng.next();
        }
        const double mu = 2.0 * rng.next() - 1.0;
        const double phi = 2.0 * M_PI * rng.next();
        const double st = sqrt(fmax(0.0, 1.0 - mu * mu));
        double sp, cp;
        sincos(phi, &sp, &cp);
        u = st * cp; v = st * sp; w = mu;
    }
    int32_t cell;
    bool inside;
    locate_point(g, x, y, cell, inside);
    b.x[s] = x; b.y[s] = y; b.z[s] = z;
    b.u[s] = u; b.v[s] = v; b.w[s] = w;
    b.E[s] = g.src_E;
    b.wt[s] = 1.0;
    b.cell[s] = cell;
    b.inside[s] = inside ? 1 : 0;
    b.mat[s] = region_material(g, cell, inside);
    b.pid[s] = pid;
    b.ndraw[s] = rng.n;
    b.lineage[s] = 0u;
    b.ncoll[s] = 0;
    b.ncross[s] = 0;
    b.track[s] = 0.0;
    b.flags[s] = F_ALIVE | F_LOOKUP;
}

__global__ void __launch_bounds__(WG) k_slots_queue(BankDev bank, GeomDev geom, Counters *ctr,
                                                    int cur, uint64_t first_pid, uint64_t n_hist,
                                                    uint64_t seed)
{
    __shared__ uint32_t lds[32];
    const uint32_t n_tiles = (bank.C + TILE - 1) / TILE;
    uint32_t pre[3], tot[3];
    tile_prefix3(bank.tile_cnt, n_tiles, blockIdx.x, lds, pre, tot);
    const Counters prev = ctr[cur ^ 1];
    const uint64_t remaining = n_hist - prev.issued;
    const uint32_t n_new = (uint32_t)((uint64_t)tot[2] < remaining ? (uint64_t)tot[2] : remaining);
    const uint32_t base = blockIdx.x * (uint32_t)TILE;
    uint32_t run[3] = {0, 0, 0};
    for (int r = 0; r < TILE_ITEMS; ++r) {
        const uint32_t s = base + r * WG + threadIdx.x;
        const bool valid = s < bank.C;
        const uint8_t f = valid ? bank.flags[s] : 0;
        const bool alive = valid && (f & F_ALIVE);
        const bool look = valid && (f & F_LOOKUP);
        const bool fr = valid && !(f & F_ALIVE);
        const Rank3 rk = block_rank3(alive, look, fr, lds);
        if (alive) bank.A[pre[0] + run[0] + rk.rank[0]] = s;
        if (look) bank.L[pre[1] + run[1] + rk.rank[1]] = s;
        if (fr) {
            const uint32_t k = pre[2] + run[2] + rk.rank[2];
            if (k < n_new) {
                init_particle(bank, geom, s, first_pid + prev.issued + k, seed);
                bank.A[tot[0] + k] = s;
                bank.L[tot[1] + k] = s;
            }
        }
#pragma unroll
        for (int q = 0; q < 3; ++q) run[q] += rk.total[q];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        Counters c;
        c.issued = prev.issued + n_new;
        c.nA = tot[0] + n_new;
        c.nL = tot[1] + n_new;
        c.nC = 0;
        c.nX = 0;
        c.n_new = n_new;
        c.pad = 0;
        ctr[cur] = c;
    }
}

// ---------------------------------------------------------------------------
// sort of the lookup queue by key = material * M + hash bin (counting sort:
// histogram, exclusive scan, scatter).  Equal keys may land in any order;
// every lookup writes only its own particle, so results do not depend on it.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(WG) k_sort_hist(XsDev xs, const uint32_t *list, const uint32_t *n_ptr,
                                                  uint32_t n_fixed, const double *E, const int32_t *mat,
                                                  uint32_t *keys, uint32_t *hist)
{
    const uint32_t n = n_ptr ? *n_ptr : n_fixed;
    const uint32_t i = blockIdx.x * WG + threadIdx.x;
    if (i >= n) return;
    const uint32_t p = list ? list[i] : i;
    int32_t m = mat[p];
    m = m < 0 ? 0 : (m >= xs.n_mat ? xs.n_mat - 1 : m);  // ids are validated by the caller; stay in bounds
    const uint32_t key = (uint32_t)m * (uint32_t)xs.M + (uint32_t)hash_bin(xs, E[p]);
    keys[i] = key;
    atomicAdd(hist + key, 1u);
}

// Exclusive scan of the histogram into offsets, zeroing the histogram for the
// next use (one workgroup of 1024 threads).
__global__ void __launch_bounds__(1024) k_sort_scan(uint32_t *hist, uint32_t *offs, uint32_t n_keys)
{
    __shared__ uint32_t part[1024];
    const uint32_t per = (n_keys + 1023u) / 1024u;
    const uint32_t lo = threadIdx.x * per;
    const uint32_t hi = lo + per < n_keys ? lo + per : n_keys;
    uint32_t s = 0;
    for (uint32_t k = lo; k < hi; ++k) s += hist[k];
    part[threadIdx.x] = s;
    __syncthreads();
    for (uint32_t o = 1; o < 1024; o <<= 1) {
        const uint32_t v = threadIdx.x >= o ? part[threadIdx.x - o] : 0u;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = part[threadIdx.x] - s;
    for (uint32_t k = lo; k < hi; ++k) {
        const uint32_t c = hist[k];
        offs[k] = run;
        run += c;
        hist[k] = 0u;
    }
}

__global__ void __launch_bounds__(WG) k_sort_scatter(const uint32_t *list, const uint32_t *n_ptr,
                                                     uint32_t n_fixed, const uint32_t *keys, uint32_t *offs,
                                                     uint32_t *out_list, uint32_t *out_keys)
{
    const uint32_t n = n_ptr ? *n_ptr : n_fixed;
    const uint32_t i = blockIdx.x * WG + threadIdx.x;
    if (i >= n) return;
    const uint32_t key = keys[i];
    const uint32_t pos = atomicAdd(offs + key, 1u);
    out_list[pos] = list ? list[i] : i;
    if (out_keys) out_keys[pos] = key;
}

// ---------------------------------------------------------------------------
// macroscopic lookup
// ---------------------------------------------------------------------------
// Lookup of queue entries [blockIdx.x*256, ...): particle p = list[i] (or i),
// energy E[p], material mat[p]; writes Sa[p], Ss[p] and clears F_LOOKUP.
// When the queue is sorted (keys != null) and the workgroup's 256 entries share
// one material and span few hash bins, the workgroup stages those bins' hash
// rows in LDS once and every lane reads its bracket from there.
struct LookupArgs {
    XsDev xs;
    const uint32_t *list;     // nullable: identity
    const uint32_t *keys;     // nullable: compute bins from E
    const uint32_t *n_ptr;    // nullable: use n_fixed
    uint32_t n_fixed;
    const double *E;
    const int32_t *mat;
    double *Sa, *Ss;
    uint8_t *flags;           // nullable
    int32_t *idx_out;         // nullable, per nuclide [p * nk + q]
    double *sc_out, *ss_out;  // nullable, per nuclide
    unsigned long long *nuc_count;  // nullable: adds sum of nk over the queue
};

constexpr int LDS_HASH_WORDS = 4096;  // 16 KiB of staged hash bounds

__global__ void __launch_bounds__(WG) k_lookup(LookupArgs a)
{
    __shared__ uint32_t sh[LDS_HASH_WORDS];
    __shared__ int32_t s_info[4];
    const XsDev &xs = a.xs;
    const uint32_t n = a.n_ptr ? *a.n_ptr : a.n_fixed;
    const uint32_t i0 = blockIdx.x * WG;
    if (i0 >= n) return;
    const uint32_t i = i0 + threadIdx.x;
    const bool valid = i < n;
    const uint32_t iL = (i0 + WG - 1 < n) ? i0 + WG - 1 : n - 1;

    // workgroup-uniform staging decision
    if (threadIdx.x == 0) {
        int32_t staged = 0, m = -1, b0 = 0, nrow = 0;
        if (a.keys) {
            const uint32_t k0 = a.keys[i0], k1 = a.keys[iL];
            const int32_t m0 = (int32_t)(k0 / (uint32_t)xs.M), m1 = (int32_t)(k1 / (uint32_t)xs.M);
            if (m0 == m1) {
                const int32_t nk = xs.mat_off[m0 + 1] - xs.mat_off[m0];
                b0 = (int32_t)(k0 % (uint32_t)xs.M);
                nrow = (int32_t)(k1 % (uint32_t)xs.M) - b0 + 2;
                if (nrow * nk <= LDS_HASH_WORDS) { staged = 1; m = m0; }
            }
        }
        s_info[0] = staged; s_info[1] = m; s_info[2] = b0; s_info[3] = nrow;
    }
    __syncthreads();
    const bool staged = s_info[0] != 0;
    if (staged) {
        const int32_t m = s_info[1], b0 = s_info[2], nrow = s_info[3];
        const int32_t nk = xs.mat_off[m + 1] - xs.mat_off[m];
        const uint32_t *src = hash_row(xs, m, b0, nk);
        for (int32_t t = threadIdx.x; t < nrow * nk; t += WG) sh[t] = src[t];
        __syncthreads();
    }
    int32_t nk_done = 0;
    if (valid) {
    const uint32_t p = a.list ? a.list[i] : i;
    const double e = a.E[p];
    int32_t m, b;
    if (a.keys) {
        const uint32_t key = a.keys[i];
        m = (int32_t)(key / (uint32_t)xs.M);
        b = (int32_t)(key % (uint32_t)xs.M);
    } else {
        m = a.mat[p];
        b = hash_bin(xs, e);
    }
    if (m < 0 || m >= xs.n_mat) {  // not a material: no table access, NaN out
        if (a.Sa) a.Sa[p] = NAN;
        if (a.Ss) a.Ss[p] = NAN;
        m = -1;
    }
    if (m >= 0) {
    const int32_t q0 = xs.mat_off[m];
    const int32_t nk = xs.mat_off[m + 1] - q0;
    const uint32_t *h0;
    if (staged) h0 = sh + (b - s_info[2]) * nk;
    else h0 = hash_row(xs, m, b, nk);
    double sa = 0.0, ss = 0.0;
    for (int32_t q = 0; q < nk; ++q) {
        const MatNuc mn = xs.mnuc[q0 + q];
        const uint32_t ix = grid_find(xs.Eg + mn.off, mn.len, h0[q], h0[nk + q], e);
        double c, s;
        lerp_xs(xs, mn.off, ix, e, c, s);
        sa = sa + mn.dens * c;
        ss = ss + mn.dens * s;
        if (a.idx_out) a.idx_out[(size_t)p * nk + q] = (int32_t)ix;
        if (a.sc_out) a.sc_out[(size_t)p * nk + q] = c;
        if (a.ss_out) a.ss_out[(size_t)p * nk + q] = s;
    }
    if (a.Sa) a.Sa[p] = sa;
    if (a.Ss) a.Ss[p] = ss;
    if (a.flags) a.flags[p] = F_ALIVE;
    nk_done = nk;
    }
    }
    if (a.nuc_count) {
        const uint32_t c = wave_sum_u32((uint32_t)nk_done);
        if (lane_id() == 0 && c) atomicAdd(a.nuc_count, (unsigned long long)c);
    }
}

// ---------------------------------------------------------------------------
// tallies: deterministic per-workgroup accumulation
// ---------------------------------------------------------------------------
// Adds val into bin `bin` (< 0: nothing) of the workgroup's row.  Each wave
// peels off one distinct bin at a time: the lanes holding it are summed by the
// butterfly and the first of them adds the sum into the wave's LDS slab; the
// four slabs are then added in wave order into the workgroup's row.
__device__ void wg_bin_add(int32_t bin, double val, double *slab, int32_t nbins, double *row)
{
    for (int32_t t = threadIdx.x; t < WAVES * nbins; t += WG) slab[t] = 0.0;
    __syncthreads();
    const int wave = threadIdx.x >> 6;
    bool active = bin >= 0;
    uint64_t mask = __ballot(active);
    while (mask) {
        const int leader = __ffsll((long long)mask) - 1;
        const int32_t B = __shfl(bin, leader, 64);
        const bool mine = active && bin == B;
        const double s = wave_sum(mine ? val : 0.0);
        if (lane_id() == leader) slab[wave * nbins + B] += s;
        active = active && !mine;
        mask = __ballot(active);
    }
    __syncthreads();
    for (int32_t t = threadIdx.x; t < nbins; t += WG) {
        double s = 0.0;
        for (int w = 0; w < WAVES; ++w) s = s + slab[w * nbins + t];
        if (s != 0.0) row[t] = row[t] + s;
    }
    __syncthreads();
}

// Adds NG per-thread values into the workgroup's global-tally row.
template <int NG>
__device__ void wg_glob_add(const int32_t (&slot)[NG], const double (&val)[NG], double *lds, double *row)
{
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NG; ++k) {
        const double s = wave_sum(val[k]);
        if (lane_id() == 0) lds[k * WAVES + wave] = s;
    }
    __syncthreads();
    if (threadIdx.x < NG) {
        double s = 0.0;
        for (int w = 0; w < WAVES; ++w) s = s + lds[threadIdx.x * WAVES + w];
        if (s != 0.0) row[slot[threadIdx.x]] = row[slot[threadIdx.x]] + s;
    }
    __syncthreads();
}

__device__ __forceinline__ int32_t energy_bin(const GeomDev &g, double e)
{
    const int32_t n = g.n_ebins;
    if (!(e >= g.e_edges[0]) || e > g.e_edges[n]) return -1;
    int32_t lo = 0, hi = n - 1;  // largest b in [0, n-1] with edge[b] <= e
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (g.e_edges[mid] <= e) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int32_t mesh_index(const GeomDev &g, double x, double y, double z)
{
    const double r[3] = {x, y, z};
    int32_t c[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (r[k] < g.mesh_lo[k] || r[k] > g.mesh_hi[k]) return -1;
        int32_t v = (int32_t)floor((r[k] - g.mesh_lo[k]) / (g.mesh_hi[k] - g.mesh_lo[k]) * g.mesh_dims[k]);
        c[k] = v > g.mesh_dims[k] - 1 ? g.mesh_dims[k] - 1 : v;
    }
    return (c[2] * g.mesh_dims[1] + c[1]) * g.mesh_dims[0] + c[0];
}

// Track-length score of a straight flight through the mesh: walk the cells it
// crosses (3-D digital differential analyser), adding w * length per cell.
__device__ void mesh_flight(const GeomDev &g, double *acc, double x, double y, double z, double u,
                            double v, double w, double d, double wt)
{
    const double r0[3] = {x, y, z}, dir[3] = {u, v, w};
    double h[3], tnext[3], tdelta[3];
    int32_t c[3], step[3];
    // start cell: the one holding the flight's first point (nudged along the
    // flight by a hair so a start on a mesh plane picks the cell ahead)
    for (int k = 0; k < 3; ++k) {
        h[k] = (g.mesh_hi[k] - g.mesh_lo[k]) / g.mesh_dims[k];
        double p = r0[k] + dir[k] * fmin(d, 1e-9) * 0.5;
        int32_t v0 = (int32_t)floor((p - g.mesh_lo[k]) / h[k]);
        c[k] = v0 < 0 ? 0 : (v0 > g.mesh_dims[k] - 1 ? g.mesh_dims[k] - 1 : v0);
        if (dir[k] > 0.0) {
            step[k] = 1;
            tnext[k] = (g.mesh_lo[k] + (c[k] + 1) * h[k] - r0[k]) / dir[k];
            tdelta[k] = h[k] / dir[k];
        } else if (dir[k] < 0.0) {
            step[k] = -1;
            tnext[k] = (g.mesh_lo[k] + c[k] * h[k] - r0[k]) / dir[k];
            tdelta[k] = -h[k] / dir[k];
        } else {
            step[k] = 0;
            tnext[k] = INFINITY;
            tdelta[k] = INFINITY;
        }
    }
    double t = 0.0;
    for (int guard = 0; guard < 100000 && t < d; ++guard) {
        int k = 0;
        if (tnext[1] < tnext[k]) k = 1;
        if (tnext[2] < tnext[k]) k = 2;
        const double t1 = fmin(fmax(tnext[k], t), d);
        if (t1 > t) {
            const int32_t idx = (c[2] * g.mesh_dims[1] + c[1]) * g.mesh_dims[0] + c[0];
            atomicAdd(acc + idx, wt * (t1 - t));
        }
        t = t1;
        if (t >= d) break;
        c[k] += step[k];
        if (c[k] < 0 || c[k] >= g.mesh_dims[k]) break;
        tnext[k] += tdelta[k];
    }
}

// ---------------------------------------------------------------------------
// advance: sample the flight, move, score track length
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(WG) k_advance(BankDev b, GeomDev g, TallyDev tal, const Counters *ctr,
                                                uint64_t seed, int64_t max_events, int32_t log_on)
{
    extern __shared__ double slab[];
    __shared__ double gl[4 * WAVES];
    const uint32_t n = ctr->nA;
    const uint32_t i0 = blockIdx.x * WG;
    if (i0 >= n) return;
    const uint32_t i = i0 + threadIdx.x;
    const bool valid = i < n;
    int32_t bin = -1;
    double val = 0.0, g_track = 0.0, g_tabs = 0.0;
    if (valid) {
        const uint32_t s = b.A[i];
        if ((int64_t)b.ncoll[s] + b.ncross[s] >= max_events) {
            // event cap reached: handled by the cross kernel as a lost particle
            b.event[s] = 0xFF;
        } else {
            double x = b.x[s], y = b.y[s], z = b.z[s];
            const double u = b.u[s], v = b.v[s], w = b.w[s];
            const double e = b.E[s], wt = b.wt[s], sa = b.Sa[s], st = sa + b.Ss[s];
            const int32_t cell = b.cell[s];
            const bool inside = b.inside[s] != 0;
            Rng rng(seed, b.pid[s], b.lineage[s], b.ndraw[s]);
            const double dc = -log(rng.next()) / st;
            uint8_t ev;
            const double db = surface_distance(g, x, y, z, u, v, w, cell, inside, ev);
            const double d = (db < dc) ? db : dc;
            if (!(db < dc)) ev = EV_COLLIDE;
            const double x0 = x, y0 = y, z0 = z;
            x = x + d * u;
            y = y + d * v;
            z = z + d * w;
            b.x[s] = x; b.y[s] = y; b.z[s] = z;
            b.ndraw[s] = rng.n;
            b.event[s] = ev;
            if (log_on) b.track[s] = b.track[s] + d;
            g_track = wt * d;
            g_tabs = wt * d * sa;
            if (tal.enabled) {
                switch (g.tally_kind) {
                case TALLY_ENERGY: bin = energy_bin(g, e); break;
                case TALLY_PIN: bin = inside ? cell : -1; break;
                case TALLY_SLAB: bin = cell; break;
                case TALLY_MESH: mesh_flight(g, tal.mesh_tl, x0, y0, z0, u, v, w, d, wt); break;
                }
                val = wt * d;
            }
        }
    }
    if (tal.enabled && g.tally_kind != TALLY_MESH)
        wg_bin_add(bin, val, slab, tal.n_bins, tal.tl + (size_t)blockIdx.x * tal.n_bins);
    const int32_t slots[2] = {G_TRACK, G_TRACK_ABS};
    const double vals[2] = {g_track, g_tabs};
    wg_glob_add<2>(slots, vals, gl, tal.glob + (size_t)blockIdx.x * N_GLOBAL);
}

// ---------------------------------------------------------------------------
// split the alive queue into collide / cross queues (stable)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(WG) k_split_count(BankDev b, const Counters *ctr)
{
    __shared__ uint32_t lds[32];
    const uint32_t n = ctr->nA;
    const uint32_t base = blockIdx.x * (uint32_t)TILE;
    uint32_t cc = 0, cx = 0;
    if (base < n) {
        for (int r = 0; r < TILE_ITEMS; ++r) {
            const uint32_t i = base + r * WG + threadIdx.x;
            if (i < n) {
                const uint8_t ev = b.event[b.A[i]];
                cc += ev == EV_COLLIDE ? 1u : 0u;
                cx += ev != EV_COLLIDE ? 1u : 0u;
            }
        }
    }
    block_count3(cc, cx, 0u, lds, b.tile_cnt + blockIdx.x * 3);
}

__global__ void __launch_bounds__(WG) k_split_scatter(BankDev b, Counters *ctr)
{
    __shared__ uint32_t lds[32];
    const uint32_t n = ctr->nA;
    const uint32_t n_tiles = (n + TILE - 1) / TILE;
    if (blockIdx.x >= n_tiles && !(blockIdx.x == 0)) return;
    uint32_t pre[3], tot[3];
    tile_prefix3(b.tile_cnt, n_tiles, blockIdx.x, lds, pre, tot);
    const uint32_t base = blockIdx.x * (uint32_t)TILE;
    uint32_t run[3] = {0, 0, 0};
    for (int r = 0; r < TILE_ITEMS; ++r) {
        const uint32_t i = base + r * WG + threadIdx.x;
        const bool valid = i < n;
        const uint32_t s = valid ? b.A[i] : 0u;
        const uint8_t ev = valid ? b.event[s] : 0;
        const bool pc = valid && ev == EV_COLLIDE;
        const bool px = valid && ev != EV_COLLIDE;
        const Rank3 rk = block_rank3(pc, px, false, lds);
        if (pc) b.Qc[pre[0] + run[0] + rk.rank[0]] = s;
        if (px) b.Qx[pre[1] + run[1] + rk.rank[1]] = s;
        run[0] += rk.total[0];
        run[1] += rk.total[1];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctr->nC = tot[0];
        ctr->nX = tot[1];
    }
}

// ---------------------------------------------------------------------------
// surface crossing
// ---------------------------------------------------------------------------
__device__ __forceinline__ void write_log(const BankDev &b, HistLog *log, uint64_t first_pid,
                                          uint32_t s, int32_t fate, double e)
{
    HistLog h;
    h.fate = fate;
    h.n_coll = b.ncoll[s];
    h.n_cross = b.ncross[s];
    h.pad = 0;
    h.n_draws = b.ndraw[s];
    h.E_final = e;
    h.track = b.track[s];
    h.weight = b.wt[s];
    log[b.pid[s] - first_pid] = h;
}

__global__ void __launch_bounds__(WG) k_cross(BankDev b, GeomDev g, TallyDev tal, const Counters *ctr,
                                              HistLog *log, uint64_t first_pid,
                                              unsigned long long *lost)
{
    __shared__ double gl[4 * WAVES];
    const uint32_t n = ctr->nX;
    const uint32_t i0 = blockIdx.x * WG;
    if (i0 >= n) return;
    const uint32_t i = i0 + threadIdx.x;
    double v_cross = 0.0, v_leak = 0.0, v_lx = 0.0, v_lxu = 0.0;
    if (i < n) {
        const uint32_t s = b.Qx[i];
        const uint8_t ev = b.event[s];
        if (ev == 0xFF) {
            b.flags[s] = 0;
            atomicAdd(lost, 1ull);
            if (log) write_log(b, log, first_pid, s, FATE_LOST, b.E[s]);
        } else {
            v_cross = 1.0;
            int32_t cell = b.cell[s];
            bool inside = b.inside[s] != 0;
            const int32_t nc = b.ncross[s] + 1;
            b.ncross[s] = nc;
            int face = -1;        // outer face reached (0..5)
            double face_pos = 0.0;
            bool leaked = false;
            if (g.kind == GEOM_SLAB) {
                if (ev == EV_XHI) {
                    if (cell == g.n_layers - 1) { face = 1; face_pos = g.x_edges[g.n_layers]; }
                    else { cell += 1; b.x[s] = g.x_edges[cell]; }
                } else {
                    if (cell == 0) { face = 0; face_pos = g.x_edges[0]; }
                    else { b.x[s] = g.x_edges[cell]; cell -= 1; }
                }
            } else {
                const int32_t ci = cell % g.nx, cj = cell / g.nx;
                const double P = g.pitch;
                switch (ev) {
                case EV_CYL: inside = !inside; break;
                case EV_XHI:
                    if (ci == g.nx - 1) { face = 1; face_pos = (double)g.nx * P; }
                    else { cell += 1; b.x[s] = (double)(ci + 1) * P; }
                    break;
                case EV_XLO:
                    if (ci == 0) { face = 0; face_pos = 0.0; }
                    else { b.x[s] = (double)ci * P; cell -= 1; }
                    break;
                case EV_YHI:
                    if (cj == g.ny - 1) { face = 3; face_pos = (double)g.ny * P; }
                    else { cell += g.nx; b.y[s] = (double)(cj + 1) * P; }
                    break;
                case EV_YLO:
                    if (cj == 0) { face = 2; face_pos = 0.0; }
                    else { b.y[s] = (double)cj * P; cell -= g.nx; }
                    break;
                case EV_ZHI: face = 5; face_pos = g.z1; break;
                case EV_ZLO: face = 4; face_pos = g.z0; break;
                default: break;
                }
            }
            if (face >= 0) {
                if (g.bc[face] == BC_VACUUM) {
                    leaked = true;
                } else {
                    const int axis = face >> 1;
                    if (axis == 0) { b.u[s] = -b.u[s]; b.x[s] = face_pos; }
                    else if (axis == 1) { b.v[s] = -b.v[s]; b.y[s] = face_pos; }
                    else { b.w[s] = -b.w[s]; b.z[s] = face_pos; }
                }
            }
            if (leaked) {
                const double wt = b.wt[s];
                v_leak = wt;
                if (face == 1) {
                    v_lx = wt;
                    if (b.ncoll[s] == 0) v_lxu = wt;
                }
                b.flags[s] = 0;
                if (log) write_log(b, log, first_pid, s, FATE_LEAKED, b.E[s]);
            } else {
                const int32_t m_old = b.mat[s];
                const int32_t m_new = region_material(g, cell, inside);
                b.cell[s] = cell;
                b.inside[s] = inside ? 1 : 0;
                if (m_new != m_old) {
                    b.mat[s] = m_new;
                    b.flags[s] = F_ALIVE | F_LOOKUP;
                }
            }
        }
    }
    const int32_t slots[4] = {G_NCROSS, G_LEAK, G_LEAK_XHI, G_LEAK_XHI_UNC};
    const double vals[4] = {v_cross, v_leak, v_lx, v_lxu};
    wg_glob_add<4>(slots, vals, gl, tal.glob + (size_t)blockIdx.x * N_GLOBAL);
}

// ---------------------------------------------------------------------------
// collision: analog capture or elastic scattering off a target at rest
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(WG) k_collide(BankDev b, XsDev xs, GeomDev g, TallyDev tal,
                                                const Counters *ctr, uint64_t seed, HistLog *log,
                                                uint64_t first_pid)
{
    extern __shared__ double slab[];
    __shared__ double gl[4 * WAVES];
    const uint32_t n = ctr->nC;
    const uint32_t i0 = blockIdx.x * WG;
    if (i0 >= n) return;
    const uint32_t i = i0 + threadIdx.x;
    int32_t bin = -1;
    double val = 0.0, v_coll = 0.0, v_n = 0.0, v_abs = 0.0, v_cut = 0.0;
    if (i < n) {
        const uint32_t s = b.Qc[i];
        const double e = b.E[s], wt = b.wt[s], sa = b.Sa[s], ssig = b.Ss[s];
        const double st = sa + ssig;
        const int32_t m = b.mat[s];
        b.ncoll[s] = b.ncoll[s] + 1;
        v_n = 1.0;
        v_coll = wt / st;
        if (tal.enabled) {
            switch (g.tally_kind) {
            case TALLY_ENERGY: bin = energy_bin(g, e); break;
            case TALLY_PIN: bin = b.inside[s] ? b.cell[s] : -1; break;
            case TALLY_SLAB: bin = b.cell[s]; break;
            case TALLY_MESH: {
                const int32_t c = mesh_index(g, b.x[s], b.y[s], b.z[s]);
                if (c >= 0) atomicAdd(tal.mesh_coll + c, wt / st);
            } break;
            }
            val = wt / st;
        }
        Rng rng(seed, b.pid[s], b.lineage[s], b.ndraw[s]);
        if (rng.next() * st < sa) {
            v_abs = wt;
            b.flags[s] = 0;
            b.ndraw[s] = rng.n;
            if (log) write_log(b, log, first_pid, s, FATE_ABSORBED, e);
        } else {
            // target: first nuclide whose running sum of density * sigma_s
            // reaches xi * Sigma_s (sigma_s gathered again, material order)
            const double target = rng.next() * ssig;
            const int32_t q0 = xs.mat_off[m], nk = xs.mat_off[m + 1] - q0;
            const int32_t hb = hash_bin(xs, e);
            double cum = 0.0;
            int32_t pick = -1;
            for (int32_t q = 0; q < nk; ++q) {
                const double term = xs.mnuc[q0 + q].dens * micro_scatter(xs, m, q, nk, hb, e);
                cum = cum + term;
                if (term > 0.0) pick = q;
                if (cum >= target && term > 0.0) break;
            }
            const double A = xs.awr[xs.mat_nuc[q0 + (pick < 0 ? 0 : pick)]];
            const double mu = 2.0 * rng.next() - 1.0;
            const double phi = 2.0 * M_PI * rng.next();
            double e2, mul;
            elastic_at_rest(A, e, mu, e2, mul);
            double u = b.u[s], v = b.v[s], w = b.w[s];
            turn(u, v, w, mul, phi);
            b.u[s] = u; b.v[s] = v; b.w[s] = w;
            b.E[s] = e2;
            b.ndraw[s] = rng.n;
            if (e2 < g.e_cut) {
                v_cut = wt;
                b.flags[s] = 0;
                if (log) write_log(b, log, first_pid, s, FATE_CUTOFF, e2);
            } else {
                b.flags[s] = F_ALIVE | F_LOOKUP;
            }
        }
    }
    if (tal.enabled && g.tally_kind != TALLY_MESH)
        wg_bin_add(bin, val, slab, tal.n_bins, tal.coll + (size_t)blockIdx.x * tal.n_bins);
    const int32_t slots[4] = {G_COLL_EST, G_NCOLL, G_ABSORB, G_CUTOFF};
    const double vals[4] = {v_coll, v_n, v_abs, v_cut};
    wg_glob_add<4>(slots, vals, gl, tal.glob + (size_t)blockIdx.x * N_GLOBAL);
}

// ---------------------------------------------------------------------------
// batch end: fixed-order reduction of the per-workgroup rows, batch sums
// ---------------------------------------------------------------------------
constexpr int RED_CHUNKS = 64;

// partial[c][k] = sum of rows [c*R/64, (c+1)*R/64) of column k (row order)
__global__ void __launch_bounds__(WG) k_rows_partial(const double *rows, int32_t n_rows, int32_t n_cols,
                                                     double *partial)
{
    const int32_t k = blockIdx.x * WG + threadIdx.x;
    const int32_t c = blockIdx.y;
    if (k >= n_cols) return;
    const int32_t r0 = (int32_t)((int64_t)c * n_rows / RED_CHUNKS);
    const int32_t r1 = (int32_t)((int64_t)(c + 1) * n_rows / RED_CHUNKS);
    double s = 0.0;
    for (int32_t r = r0; r < r1; ++r) s = s + rows[(size_t)r * n_cols + k];
    partial[(size_t)c * n_cols + k] = s;
}

// T = (sum of the partials in chunk order, or the atomic accumulator) / n;
// S1 += T; S2 += T^2.
__global__ void __launch_bounds__(WG) k_batch_stats(const double *partial, const double *direct,
                                                    int32_t n_cols, double inv_n, double *S1, double *S2)
{
    const int32_t k = blockIdx.x * WG + threadIdx.x;
    if (k >= n_cols) return;
    double s = 0.0;
    if (direct) {
        s = direct[k];
    } else {
        for (int c = 0; c < RED_CHUNKS; ++c) s = s + partial[(size_t)c * n_cols + k];
    }
    const double T = s * inv_n;
    S1[k] = S1[k] + T;
    S2[k] = S2[k] + T * T;
}

// ---------------------------------------------------------------------------
// host-side launch wrappers
// ---------------------------------------------------------------------------
static inline unsigned blocks_for(size_t n, size_t per) { return (unsigned)((n + per - 1) / per); }

// LDS of the per-wave tally slabs (none when the binned tallies are off or
// use the mesh path)
static inline size_t slab_bytes(const GeomDev &g, const TallyDev &t)
{
    if (!t.enabled || g.tally_kind == TALLY_MESH) return 0;
    return (size_t)WAVES * (size_t)t.n_bins * sizeof(double);
}

hipError_t launch_fill_u8(uint8_t *p, size_t n, uint8_t v, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    unsigned g = blocks_for(n, WG);
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_fill_u8, dim3(g), dim3(WG), 0, st, p, n, v);
    return hipGetLastError();
}
hipError_t launch_fill_u32(uint32_t *p, size_t n, uint32_t v, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    unsigned g = blocks_for(n, WG);
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3(g), dim3(WG), 0, st, p, n, v);
    return hipGetLastError();
}
hipError_t launch_fill_f64(double *p, size_t n, double v, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    unsigned g = blocks_for(n, WG);
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_fill_f64, dim3(g), dim3(WG), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_slots_count(const BankDev &b, hipStream_t st)
{
    hipLaunchKernelGGL(k_slots_count, dim3(blocks_for(b.C, TILE)), dim3(WG), 0, st, b);
    return hipGetLastError();
}

hipError_t launch_slots_queue(const BankDev &b, const GeomDev &g, Counters *ctr, int cur,
                              uint64_t first_pid, uint64_t n_hist, uint64_t seed, hipStream_t st)
{
    hipLaunchKernelGGL(k_slots_queue, dim3(blocks_for(b.C, TILE)), dim3(WG), 0, st, b, g, ctr, cur,
                       first_pid, n_hist, seed);
    return hipGetLastError();
}

hipError_t launch_sort(const XsDev &xs, const uint32_t *list, const uint32_t *n_ptr, uint32_t n_bound,
                       const double *E, const int32_t *mat, uint32_t *keys_tmp, uint32_t *hist,
                       uint32_t *offs, uint32_t n_keys, uint32_t *out_list, uint32_t *out_keys,
                       hipStream_t st)
{
    if (n_bound == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sort_hist, dim3(blocks_for(n_bound, WG)), dim3(WG), 0, st, xs, list, n_ptr,
                       n_bound, E, mat, keys_tmp, hist);
    hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(1024), 0, st, hist, offs, n_keys);
    hipLaunchKernelGGL(k_sort_scatter, dim3(blocks_for(n_bound, WG)), dim3(WG), 0, st, list, n_ptr,
                       n_bound, keys_tmp, offs, out_list, out_keys);
    return hipGetLastError();
}

hipError_t launch_lookup(const LookupLaunch &l, hipStream_t st)
{
    if (l.n_bound == 0) return hipSuccess;
    LookupArgs a;
    a.xs = l.xs;
    a.list = l.list;
    a.keys = l.keys;
    a.n_ptr = l.n_ptr;
    a.n_fixed = l.n_bound;
    a.E = l.E;
    a.mat = l.mat;
    a.Sa = l.Sa;
    a.Ss = l.Ss;
    a.flags = l.flags;
    a.idx_out = l.idx_out;
    a.sc_out = l.sc_out;
    a.ss_out = l.ss_out;
    a.nuc_count = l.nuc_count;
    hipLaunchKernelGGL(k_lookup, dim3(blocks_for(l.n_bound, WG)), dim3(WG), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_advance(const BankDev &b, const GeomDev &g, const TallyDev &t, const Counters *ctr,
                          uint32_t n_bound, uint64_t seed, int64_t max_events, int32_t log_on,
                          hipStream_t st)
{
    if (n_bound == 0) return hipSuccess;
    const size_t lds = slab_bytes(g, t);
    hipLaunchKernelGGL(k_advance, dim3(blocks_for(n_bound, WG)), dim3(WG), lds, st, b, g, t, ctr, seed,
                       max_events, log_on);
    return hipGetLastError();
}

hipError_t launch_split(const BankDev &b, Counters *ctr, uint32_t n_bound, hipStream_t st)
{
    const unsigned nt = blocks_for(n_bound > 0 ? n_bound : 1, TILE);
    hipLaunchKernelGGL(k_split_count, dim3(nt), dim3(WG), 0, st, b, ctr);
    hipLaunchKernelGGL(k_split_scatter, dim3(nt), dim3(WG), 0, st, b, ctr);
    return hipGetLastError();
}

hipError_t launch_cross(const BankDev &b, const GeomDev &g, const TallyDev &t, const Counters *ctr,
                        uint32_t n_bound, HistLog *log, uint64_t first_pid, unsigned long long *lost,
                        hipStream_t st)
{
    if (n_bound == 0) return hipSuccess;
    hipLaunchKernelGGL(k_cross, dim3(blocks_for(n_bound, WG)), dim3(WG), 0, st, b, g, t, ctr, log,
                       first_pid, lost);
    return hipGetLastError();
}

hipError_t launch_collide(const BankDev &b, const XsDev &xs, const GeomDev &g, const TallyDev &t,
                          const Counters *ctr, uint32_t n_bound, uint64_t seed, HistLog *log,
                          uint64_t first_pid, hipStream_t st)
{
    if (n_bound == 0) return hipSuccess;
    const size_t lds = slab_bytes(g, t);
    hipLaunchKernelGGL(k_collide, dim3(blocks_for(n_bound, WG)), dim3(WG), lds, st, b, xs, g, t, ctr, seed,
                       log, first_pid);
    return hipGetLastError();
}

hipError_t launch_batch_stats(const double *rows, int32_t n_rows, int32_t n_cols, const double *direct,
                              double *partial, double inv_n, double *S1, double *S2, hipStream_t st)
{
    if (n_cols == 0) return hipSuccess;
    if (!direct) {
        hipLaunchKernelGGL(k_rows_partial, dim3(blocks_for(n_cols, WG), RED_CHUNKS), dim3(WG), 0, st, rows,
                           n_rows, n_cols, partial);
    }
    hipLaunchKernelGGL(k_batch_stats, dim3(blocks_for(n_cols, WG)), dim3(WG), 0, st, partial, direct,
                       n_cols, inv_n, S1, S2);
    return hipGetLastError();
}

}  // namespace mc
