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
#include "mc_physics.h"
#include "mc_ww.h"

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
// queue building over the slots (one tile of TILE slots per workgroup)
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
__device__ __forceinline__ void init_particle(const BankDev &b, const GeomDev &g, const WwDev &W, uint32_t s,
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
    ww_start(W, s, x, g.src_E);
}

// Copy q of the copy bank into slot s: a weight-window copy starting with its
// own stream at draw 0, a path length of 0, its parent's counts, cells and
// split generation; lookup due.
__device__ __forceinline__ void load_copy(const BankDev &b, const WwDev &W, uint32_t s, uint32_t q)
{
    b.x[s] = W.qx[q]; b.y[s] = W.qy[q]; b.z[s] = W.qz[q];
    b.u[s] = W.qu[q]; b.v[s] = W.qv[q]; b.w[s] = W.qw[q];
    b.E[s] = W.qE[q]; b.wt[s] = W.qwt[q];
    b.cell[s] = W.qcell[q]; b.mat[s] = W.qmat[q]; b.inside[s] = W.qinside[q];
    b.ncoll[s] = W.qncoll[q]; b.ncross[s] = W.qncross[q];
    b.pid[s] = W.qpid[q];
    b.lineage[s] = W.qlin[q];
    b.ndraw[s] = 0u;
    b.track[s] = 0.0;
    b.flags[s] = F_ALIVE | F_LOOKUP;
    W.depth_of[s] = 0;
    W.splits[s] = 0;
    W.gen[s] = W.qgen[q];
    W.inh_coll[s] = W.qncoll[q];
    W.inh_cross[s] = W.qncross[q];
    if (W.imp_nx) {
        for (int32_t e = 0; e < W.imp_ne; ++e) W.iv[(size_t)e * W.C + s] = W.qiv[(size_t)e * W.Q + q];
    }
}

__global__ void __launch_bounds__(WG) k_slots_queue(BankDev bank, GeomDev geom, WwDev W, Counters *ctr,
                                                    int cur, uint64_t first_pid, uint64_t n_hist,
                                                    uint64_t seed)
{
    __shared__ uint32_t lds[32];
    const uint32_t n_tiles = (bank.C + TILE - 1) / TILE;
    uint32_t pre[3], tot[3];
    tile_prefix3(bank.tile_cnt, n_tiles, blockIdx.x, lds, pre, tot);
    const Counters prev = ctr[cur ^ 1];
    const uint64_t remaining = n_hist - prev.issued;
    // free slots take waiting weight-window copies first, then new histories
    const uint32_t qtop = prev.top_after;
    const uint32_t n_copy = tot[2] < qtop ? tot[2] : qtop;
    const uint32_t n_free = tot[2] - n_copy;
    const uint32_t n_new = (uint32_t)((uint64_t)n_free < remaining ? (uint64_t)n_free : remaining);
    const uint32_t base = blockIdx.x * (uint32_t)TILE;
    const uint32_t n_refill = n_copy + n_new;  // the first n_refill free slots are refilled
    uint32_t run[3] = {0, 0, 0};
    // every item's flags loaded before any queue entry is stored (a load
    // waits for the earlier stores of its wave)
    uint8_t fl[TILE_ITEMS];
#pragma unroll
    for (int r = 0; r < TILE_ITEMS; ++r) {
        const uint32_t s = base + r * WG + threadIdx.x;
        fl[r] = s < bank.C ? bank.flags[s] : 0;
    }
    for (int r = 0; r < TILE_ITEMS; ++r) {
        const uint32_t s = base + r * WG + threadIdx.x;
        const bool valid = s < bank.C;
        const uint8_t f = fl[r];
        const bool alive = valid && (f & F_ALIVE);
        const bool look = valid && (f & F_LOOKUP);
        const bool fr = valid && !(f & F_ALIVE);
        const Rank3 rk = block_rank3(alive, look, fr, lds);
        // the queues hold their slots in slot order, refilled ones included:
        // slot s follows the alive (lookup) slots and the refilled slots
        // before it, so with every slot alive the alive queue is the identity
        const uint32_t k = pre[2] + run[2] + rk.rank[2];  // free slots before s
        const uint32_t ref = k < n_refill ? k : n_refill;  // refilled slots before s
        const uint32_t ia = pre[0] + run[0] + rk.rank[0] + ref, il = pre[1] + run[1] + rk.rank[1] + ref;
        if (alive) bank.A[ia] = s;
        if (look) bank.L[il] = s;
        if (fr && k < n_refill) {
            // copies load here; new histories start in k_slots_init, from the
            // list of their slots (the cross queue is free until the split)
            if (k < n_copy) load_copy(bank, W, s, qtop - 1u - k);
            else bank.Qx[k - n_copy] = s;
            bank.A[ia] = s;
            bank.L[il] = s;
        }
#pragma unroll
        for (int q = 0; q < 3; ++q) run[q] += rk.total[q];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        Counters c;
        c.issued = prev.issued + n_new;
        c.nA = tot[0] + n_copy + n_new;
        c.nL = tot[1] + n_copy + n_new;
        c.nC = 0;
        c.nX = 0;
        c.n_new = n_new;
        c.top = qtop - n_copy;
        c.top_after = qtop - n_copy;
        c.pad = 0;
        ctr[cur] = c;
    }
}

// The source particles the refill started: the j-th new history of this
// iteration (pid first_pid + issued - n_new + j) in slot Qx[j].  Its own
// kernel, so that the queue scan runs without the source sampling's registers.
__global__ void __launch_bounds__(WG) k_slots_init(BankDev bank, GeomDev geom, WwDev W, const Counters *ctr, int cur,
                                                   uint64_t first_pid, uint64_t seed)
{
    const Counters c = ctr[cur];
    const uint32_t j = blockIdx.x * WG + threadIdx.x;
    if (j >= c.n_new) return;
    init_particle(bank, geom, W, bank.Qx[j], first_pid + (c.issued - c.n_new) + j, seed);
}

// ---------------------------------------------------------------------------
// sort of a queue by key = material * M + hash bin of E: a stable LSD radix
// sort, 8 bits per pass.  Per pass: count the digits of each 4096-item tile
// (wave multi-split, one LDS add per distinct digit of a wave), scan the
// per-chunk digit totals, and scatter each tile in item order to
//   chunk offset + earlier tiles of the chunk + earlier waves + lane rank.
// Ranks come from ballots, not atomics, so the order is stable and the same
// run to run.
// ---------------------------------------------------------------------------
// Tiles of WG * items keys, items in [1, 16] chosen per sort so that a
// queue of a few hundred thousand keys still spreads over ~1024 workgroups;
// chunks of at least 16 tiles, at most 128 chunks for the one-workgroup scan.
// The kernels take the shape from the queue's length as they read it on the
// device, so a launch sized for a bound sorts a shorter queue as if it had
// been sized for it.
struct SortShape {
    uint32_t items, tiles, chunk, chunks;
};
constexpr uint32_t SORT_BATCH = 4;  // items of a thread loaded together

__host__ __device__ inline SortShape sort_shape(uint32_t n)
{
    SortShape s;
    const uint32_t per = 1024u * WG;
    s.items = (n + per - 1) / per;
    s.items = s.items < 1u ? 1u : (s.items > 16u ? 16u : s.items);
    const uint32_t tile = s.items * WG;
    s.tiles = (n + tile - 1) / tile;
    s.chunk = (s.tiles + 127u) / 128u;
    s.chunk = s.chunk < 16u ? 16u : s.chunk;
    s.chunks = (s.tiles + s.chunk - 1) / s.chunk;
    return s;
}

// Lanes of the wave holding the same 8-bit digit (0 for an invalid lane).
__device__ __forceinline__ uint64_t digit_peers(uint32_t d, bool valid)
{
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bb = __ballot(bit);
        m &= bit ? bb : ~bb;
    }
    return valid ? m : 0ull;
}

__device__ __forceinline__ uint32_t sort_key(const XsDev &xs, const double *E, const int32_t *mat, uint32_t p)
{
    int32_t m = mat[p];
    m = m < 0 ? 0 : (m >= xs.n_mat ? xs.n_mat - 1 : m);  // ids are validated by the caller; stay in bounds
    return (uint32_t)m * (uint32_t)xs.M + (uint32_t)hash_bin(xs, E[p]);
}

struct SortPassArgs {
    XsDev xs;
    const double *E;
    const int32_t *mat;
    const uint32_t *n_ptr;
    uint32_t n_fixed;
    int32_t shift;
    const uint32_t *keys_in;   // null on the first pass: keys computed from (E, mat) of vals_in
    uint32_t *keys_first;      // first pass: where the computed keys go
    const uint32_t *vals_in;   // null: identity
    uint32_t *keys_out, *vals_out;
    uint32_t *tile_hist;       // [tiles][256]
    uint32_t *chunk_total;     // [chunks][256], zero on entry of a count
    const uint32_t *chunk_off; // [chunks + 1][256] (see k_radix_scan)
};

__global__ void __launch_bounds__(WG) k_radix_count(SortPassArgs a)
{
    __shared__ uint32_t h[256];
    const uint32_t n = a.n_ptr ? *a.n_ptr : a.n_fixed;
    const SortShape sh = sort_shape(n);
    const uint32_t base = blockIdx.x * sh.items * (uint32_t)WG;
    if (base >= n) return;
    h[threadIdx.x] = 0u;
    __syncthreads();
    // keys SORT_BATCH items at a time, all loaded before any is stored (a
    // load waits for the earlier stores of its wave)
    for (uint32_t r0 = 0; r0 < sh.items; r0 += SORT_BATCH) {
        uint32_t key[SORT_BATCH];
        bool valid[SORT_BATCH];
#pragma unroll
        for (uint32_t j = 0; j < SORT_BATCH; ++j) {
            const uint32_t i = base + (r0 + j) * WG + threadIdx.x;
            valid[j] = r0 + j < sh.items && i < n;
            key[j] = 0u;
            if (valid[j]) key[j] = a.keys_in ? a.keys_in[i] : sort_key(a.xs, a.E, a.mat, a.vals_in ? a.vals_in[i] : i);
        }
#pragma unroll
        for (uint32_t j = 0; j < SORT_BATCH; ++j) {
            if (r0 + j >= sh.items) break;  // (uniform)
            if (valid[j] && !a.keys_in) a.keys_first[base + (r0 + j) * WG + threadIdx.x] = key[j];
            const uint32_t d = (key[j] >> a.shift) & 255u;
            const uint64_t peers = digit_peers(d, valid[j]);
            if (valid[j] && lane_id() == __ffsll((long long)peers) - 1) atomicAdd(&h[d], (uint32_t)__popcll(peers));
        }
    }
    __syncthreads();
    const uint32_t c = h[threadIdx.x];
    a.tile_hist[blockIdx.x * 256 + threadIdx.x] = c;
    if (c) atomicAdd(&a.chunk_total[(blockIdx.x / sh.chunk) * 256 + threadIdx.x], c);
}

// chunk_off[c][d] = items of digit d in chunks < c, and in the row after the
// last chunk, chunk_off[n_chunks][d] = items with digit < d (the scatter adds
// the two); resets chunk_total for the next pass.  One workgroup, thread =
// digit, one pass over the chunk totals.
__global__ void __launch_bounds__(WG) k_radix_scan(uint32_t *chunk_total, uint32_t *chunk_off,
                                                   const uint32_t *n_ptr, uint32_t n_fixed)
{
    __shared__ uint32_t tot[256];
    const uint32_t n_chunks = sort_shape(n_ptr ? *n_ptr : n_fixed).chunks;
    const uint32_t d = threadIdx.x;
    constexpr uint32_t B = 16;  // chunk totals loaded together (independent loads in flight)
    uint32_t run = 0;
    for (uint32_t c0 = 0; c0 < n_chunks; c0 += B) {
        uint32_t v[B];
#pragma unroll
        for (uint32_t k = 0; k < B; ++k) v[k] = c0 + k < n_chunks ? chunk_total[(c0 + k) * 256 + d] : 0u;
#pragma unroll
        for (uint32_t k = 0; k < B; ++k) {
            if (c0 + k < n_chunks) {
                chunk_off[(c0 + k) * 256 + d] = run;
                chunk_total[(c0 + k) * 256 + d] = 0u;
            }
            run += v[k];
        }
    }
    tot[d] = run;
    __syncthreads();
    // exclusive scan over the 256 digit totals (Hillis-Steele)
    for (uint32_t o = 1; o < 256; o <<= 1) {
        const uint32_t v = d >= o ? tot[d - o] : 0u;
        __syncthreads();
        tot[d] += v;
        __syncthreads();
    }
    chunk_off[n_chunks * 256 + d] = tot[d] - run;
}

__global__ void __launch_bounds__(WG) k_radix_scatter(SortPassArgs a)
{
    __shared__ uint32_t off[256];
    __shared__ uint32_t wc[WAVES * 256];
    const uint32_t n = a.n_ptr ? *a.n_ptr : a.n_fixed;
    const SortShape sh = sort_shape(n);
    const uint32_t base = blockIdx.x * sh.items * (uint32_t)WG;
    if (base >= n) return;
    const uint32_t t = blockIdx.x, c0 = (t / sh.chunk) * sh.chunk;
    {
        uint32_t o = a.chunk_off[(t / sh.chunk) * 256 + threadIdx.x] + a.chunk_off[sh.chunks * 256 + threadIdx.x];
        // the chunk's earlier tiles, their histograms loaded 8 at a time
        for (uint32_t u0 = c0; u0 < t; u0 += 8) {
            uint32_t v[8];
#pragma unroll
            for (uint32_t k = 0; k < 8; ++k) v[k] = u0 + k < t ? a.tile_hist[(u0 + k) * 256 + threadIdx.x] : 0u;
#pragma unroll
            for (uint32_t k = 0; k < 8; ++k) o += v[k];
        }
        off[threadIdx.x] = o;
    }
    const int wave = threadIdx.x >> 6;
    const uint64_t lt = lanemask_lt();
    const uint32_t *keys_in = a.keys_in ? a.keys_in : a.keys_first;
    // SORT_BATCH items' keys and values loaded before any is scattered (a
    // load waits for the earlier stores of its wave)
    for (uint32_t r0 = 0; r0 < sh.items; r0 += SORT_BATCH) {
        uint32_t kb[SORT_BATCH], vb[SORT_BATCH];
#pragma unroll
        for (uint32_t j = 0; j < SORT_BATCH; ++j) {
            const uint32_t i = base + (r0 + j) * WG + threadIdx.x;
            const bool valid = r0 + j < sh.items && i < n;
            kb[j] = valid ? keys_in[i] : 0u;
            vb[j] = valid ? (a.vals_in ? a.vals_in[i] : i) : 0u;
        }
#pragma unroll
        for (uint32_t j = 0; j < SORT_BATCH; ++j) {
            if (r0 + j >= sh.items) break;  // (uniform)
#pragma unroll
            for (int w = 0; w < WAVES; ++w) wc[w * 256 + threadIdx.x] = 0u;
            __syncthreads();
            const bool valid = base + (r0 + j) * WG + threadIdx.x < n;
            const uint32_t key = kb[j];
            const uint32_t d = (key >> a.shift) & 255u;
            const uint64_t peers = digit_peers(d, valid);
            if (valid && lane_id() == __ffsll((long long)peers) - 1) wc[wave * 256 + d] = (uint32_t)__popcll(peers);
            __syncthreads();
            if (valid) {
                uint32_t pos = off[d] + (uint32_t)__popcll(peers & lt);
                for (int w = 0; w < wave; ++w) pos += wc[w * 256 + d];
                a.keys_out[pos] = key;
                a.vals_out[pos] = vb[j];
            }
            __syncthreads();
            uint32_t add = 0;
#pragma unroll
            for (int w = 0; w < WAVES; ++w) add += wc[w * 256 + threadIdx.x];
            off[threadIdx.x] += add;
            __syncthreads();
        }
    }
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
    double *cp;               // nullable: scattering-sum checkpoints [slot][CP_MAX]
    double *sx;               // reaction channels [p][n_chan] (the CHAN kernels)
};

constexpr int LDS_HASH_PAIRS = 2048;  // 16 KiB of staged hash brackets

// Grid points a wave stages per nuclide for a sorted queue (see window_lookups),
// and reaction-channel values (window points * channels).
constexpr int WIN_PTS = 64;
constexpr int WIN_CHAN = 512;

// Orders a wave's LDS writes before its reads of them (and reads before the
// next writes): LDS instructions of one wave execute in program order, so only
// the compiler has to be kept from moving them.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Lookups of a staged workgroup of a sorted queue: one material, hash bins
// ascending through the workgroup, bracket rows b0 .. in LDS (sh).  Per
// nuclide the lanes of a wave need grid points only from the bracket start of
// the wave's lowest bin to one past the bracket end of its highest.  When that
// window holds at most WIN_PTS points the wave reads it (energies and cross
// sections) with one coalesced load each into LDS, and every lane bisects its
// own bracket there and interpolates from there; a wider window falls back to
// each lane searching global memory.  The search in LDS starts at a guess,
// the bracket point at the lane's fractional position inside its hash bin
// (points of a bin are roughly log-uniform), and walks from there to the
// largest j of the bracket with E_j <= E: usually no step, so a nuclide costs
// one round of LDS reads instead of a bisection's chain of dependent ones.  Per nuclide a wave then issues two
// vector loads instead of one per bracket, probe and interval point.  Same
// interval (with the one-off-bin walk), interpolation and sums in material
// order as micro_group: the results bit for bit.  CHAN: the reaction
// channels are assembled from the interval found, as channel_group does; the
// window's channel rows are staged in LDS too when they fit in WIN_CHAN
// values, else each lane reads its two rows.  Returns the nuclides looked up
// for this lane.
template <bool CHAN>
__device__ __forceinline__ void window_channels(const double *r0, int32_t K, double dens, double f,
                                                double (&acc)[MAX_CHAN])
{
    const double *r1 = r0 + K;
#pragma unroll
    for (int xc = 0; xc < MAX_CHAN; ++xc)
        if (xc < K) acc[xc] = acc[xc] + dens * (r0[xc] + f * (r1[xc] - r0[xc]));
}

// A wave-uniform read of a table that no kernel writes while it runs (the
// material's nuclide rows), through the constant address space: the compiler
// then issues a scalar load, and the vector loads in flight are not waited
// for before it.
template <class T>
__device__ __forceinline__ T uniform_load(const T *p, int64_t i)
{
#if defined(__HIP_DEVICE_COMPILE__)
    typedef const T __attribute__((address_space(4))) *const_ptr;
    return ((const_ptr)p)[i];
#else  // the host pass of the single-source compile never runs this
    return p[i];
#endif
}

template <bool CHAN>
__device__ __forceinline__ int32_t window_lookups(const LookupArgs &a, const uint2 *sh, const int32_t *s_info,
                                                  uint32_t i, bool valid, double *we, double2 *wx, double *wc)
{
    const XsDev &xs = a.xs;
    const uint64_t vmask = __ballot(valid);
    if (!vmask) return 0;
    const int32_t m = __builtin_amdgcn_readfirstlane(s_info[1]);
    const int32_t b0 = __builtin_amdgcn_readfirstlane(s_info[2]);
    const int32_t q0 = __builtin_amdgcn_readfirstlane(xs.mat_off[m]);
    const int32_t nk = __builtin_amdgcn_readfirstlane(xs.mat_off[m + 1]) - q0;
    // a lane past the end of the queue works on the wave's first particle
    // (same values, never stored), so the nuclide loop needs no lane mask
    const uint32_t i_own = valid ? i : i - (uint32_t)lane_id() + (uint32_t)(__ffsll((long long)vmask) - 1);
    const uint32_t p = a.list ? a.list[i_own] : i_own;
    const double e = a.E[p];
    const int32_t b = (int32_t)(a.keys[i_own] % (uint32_t)xs.M);
    const int32_t bmin = __builtin_amdgcn_readfirstlane(__shfl(b, __ffsll((long long)vmask) - 1, 64));
    const int32_t bmax = __builtin_amdgcn_readfirstlane(__shfl(b, 63 - __clzll((long long)vmask), 64));
    const uint2 *hmin = sh + (bmin - b0) * nk, *hmax = sh + (bmax - b0) * nk, *hown = sh + (b - b0) * nk;
    const uint32_t lane = (uint32_t)lane_id();
    double *E_w = we + 1 + (threadIdx.x & ~63u);  // one pad point before and after the waves' rows
    double2 *X_w = wx + (threadIdx.x & ~63u);
    double *C_w = wc + (CHAN ? (threadIdx.x >> 6) * WIN_CHAN : 0);
    const int32_t K = CHAN ? xs.n_chan : 0;
    // the lane's position inside its hash bin, in [0, 1): a guide only (the
    // walk below decides the index), so single precision is enough
    const float tb = bin_position(xs, e, b);
    const int32_t cp_sh = a.cp && nk > CP_MIN_NUC ? cp_shift(nk) : 30;  // 30: never a checkpoint
    const int32_t cp_mask = (1 << cp_sh) - 1;
    CpPairs cpw{a.cp ? a.cp + (size_t)p * CP_MAX : nullptr, 0.0};
    double sa = 0.0, ss = 0.0;
    double acc[MAX_CHAN];
    if (CHAN) {
#pragma unroll
        for (int xc = 0; xc < MAX_CHAN; ++xc) acc[xc] = 0.0;
    }
    // nuclide q's window: first point and count (wave-uniform), and this
    // lane's point of it, loaded one nuclide ahead so that the loads of the
    // next window are in flight while the lanes search the current one
    MatNuc mn_n = uniform_load(xs.mnuc, q0);
    uint32_t wlo_n = __builtin_amdgcn_readfirstlane(hmin[0].x);
    uint32_t wn_n = __builtin_amdgcn_readfirstlane(hmax[0].y) + 2u - wlo_n;  // points wlo .. wlo + wn - 1
    double pe = 0.0;
    double2 px = make_double2(0.0, 0.0);
    if (wn_n <= (uint32_t)WIN_PTS && lane < wn_n) {
        pe = xs.Eg[mn_n.off + wlo_n + lane];
        px = xs.xs[mn_n.off + wlo_n + lane];
    }
    for (int32_t q = 0; q < nk; ++q) {
        const MatNuc mn = mn_n;
        const uint32_t wlo = wlo_n, wn = wn_n;
        const double ce = pe;
        const double2 cx = px;
        if (q + 1 < nk) {
            mn_n = uniform_load(xs.mnuc, (int64_t)q0 + q + 1);
            wlo_n = __builtin_amdgcn_readfirstlane(hmin[q + 1].x);
            wn_n = __builtin_amdgcn_readfirstlane(hmax[q + 1].y) + 2u - wlo_n;
            if (wn_n <= (uint32_t)WIN_PTS && lane < wn_n) {
                pe = xs.Eg[mn_n.off + wlo_n + lane];
                px = xs.xs[mn_n.off + wlo_n + lane];
            }
        }
        const double *g = xs.Eg + mn.off;
        const double2 *x = xs.xs + mn.off;
        double c = 0.0, sg = 0.0, f = 0.0;
        uint32_t ii = 0;
        if (wn <= (uint32_t)WIN_PTS) {
            const uint32_t nc = CHAN ? wn * (uint32_t)K : 0u;
            const bool cwin = CHAN && nc <= (uint32_t)WIN_CHAN;
            if (cwin) {  // the window's channel rows: contiguous, 4 loads per lane at a time
                const double *src = xs.xc + (size_t)(mn.off + wlo) * (size_t)K;
                for (uint32_t j0 = 0; j0 < nc; j0 += 256u) {
                    double v[4];
#pragma unroll
                    for (uint32_t r = 0; r < 4; ++r) {
                        const uint32_t j = j0 + r * 64u + lane;
                        v[r] = j < nc ? src[j] : 0.0;
                    }
#pragma unroll
                    for (uint32_t r = 0; r < 4; ++r) {
                        const uint32_t j = j0 + r * 64u + lane;
                        if (j < nc) C_w[j] = v[r];
                    }
                }
            }
            if (lane < wn) {
                E_w[lane] = ce;
                X_w[lane] = cx;
            }
            wave_lds_sync();
            {
                // largest k in the bracket [lo, hi] with E_k <= e (lo when
                // none).  The guess j (nearest to the lane's position in the
                // bin) and its neighbours are read at once: k is j - 1, j or
                // j + 1 for all but ~0.05 % of lanes, which walk on.  The
                // window holds lo .. hi + 1; E_w[j - 1] and E_w[j + 2] may
                // lie one past it (padding or a neighbour's row: then unused).
                const uint32_t lo = hown[q].x, hi = hown[q].y;
                const uint32_t j = bracket_guess(lo, hi, tb);
                const double *Ej = E_w + (int32_t)(j - wlo);
                const double em = Ej[-1], eg = Ej[0], eg1 = Ej[1], ep = Ej[2];
                const bool dn = j > lo && e < eg;
                const bool up = !dn && j < hi && e >= eg1;
                uint32_t k = dn ? j - 1u : (up ? j + 1u : j);
                double e0 = dn ? em : (up ? eg1 : eg);
                double e1 = dn ? eg : (up ? ep : eg1);
                // rare: the interval lies further than one step from the
                // guess, or outside the bracket (the hash bin computed one off
                // at a bin edge).  A wave-uniform test, so the common case
                // skips the walks without any lane masking.
                const bool rare = (k > 0u && e < e0) || (k + 2u < mn.len && e >= e1);
                bool glob = false;
                if (__ballot(rare)) {
                    if (rare) {
                        while (k > lo && e < e0) {
                            --k;
                            e1 = e0;
                            e0 = E_w[k - wlo];
                        }
                        while (k < hi && e >= e1) {
                            ++k;
                            e0 = e1;
                            e1 = E_w[k + 1u - wlo];
                        }
                        glob = (e < e0 && k > 0u) || (e >= e1 && k + 2u < mn.len);
                    }
                }
                // k lies in the bracket, inside the window: the cross sections
                // from LDS; a lane whose hash bin was computed one off then
                // walks to the defined index in global memory and reloads
                double2 x0 = X_w[k - wlo], x1 = X_w[k + 1u - wlo];
                if (__ballot(glob)) {
                    if (glob) {
                        while (k > 0u && e < g[k]) --k;
                        while (k + 2u < mn.len && e >= g[k + 1u]) ++k;
                        e0 = g[k];
                        e1 = g[k + 1u];
                        x0 = x[k];
                        x1 = x[k + 1u];
                    }
                }
                ii = k;
                f = (e - e0) / (e1 - e0);
                c = x0.x + f * (x1.x - x0.x);
                sg = x0.y + f * (x1.y - x0.y);
                if (CHAN) {
                    if (cwin && ii >= wlo && ii + 1u < wlo + wn)
                        window_channels<CHAN>(C_w + (size_t)(ii - wlo) * (size_t)K, K, mn.dens, f, acc);
                    else
                        window_channels<CHAN>(xs.xc + (size_t)(mn.off + ii) * (size_t)K, K, mn.dens, f, acc);
                }
            }
            wave_lds_sync();
        } else {
            ii = grid_find(g, mn.len, hown[q].x, hown[q].y, e);
            const double e0 = g[ii], e1 = g[ii + 1u];
            const double2 x0 = x[ii], x1 = x[ii + 1u];
            f = (e - e0) / (e1 - e0);
            c = x0.x + f * (x1.x - x0.x);
            sg = x0.y + f * (x1.y - x0.y);
            if (CHAN) window_channels<CHAN>(xs.xc + (size_t)(mn.off + ii) * (size_t)K, K, mn.dens, f, acc);
        }
        sa = sa + mn.dens * c;
        ss = ss + mn.dens * sg;
        // (a lane past the queue's end writes the same values as the lane
        // whose particle it repeats, into that particle's row)
        const int32_t done = q + 1;
        if ((done & cp_mask) == 0) cpw.put((done >> cp_sh) - 1, ss);
    }
    if (!valid) return 0;
    if (cp_sh != 30) cpw.finish(nk >> cp_sh);
    if (a.Sa) a.Sa[p] = sa;
    if (a.Ss) a.Ss[p] = ss;
    if (CHAN) {
#pragma unroll
        for (int xc = 0; xc < MAX_CHAN; ++xc)
            if (xc < xs.n_chan) a.sx[(size_t)p * xs.n_chan + xc] = acc[xc];
    }
    if (a.flags) a.flags[p] = F_ALIVE;
    return nk;
}

// One nuclide's search in window_search: its grid window (points wlo ..,
// staged at Ew / Xw; the window holds lo .. hi + 1), this lane's hash
// bracket [lo, hi], its tables g / x in global memory and its grid length.
struct WinQ {
    const double *Ew;
    const double2 *Xw;
    uint32_t wlo, lo, hi, len;
    const double *g;
    const double2 *x;
};

// The interval's energies and cross sections.
struct WinHit {
    double e0, e1;
    double2 x0, x1;
};

// Interval i(E) of each of N nuclides (side by side, so that their LDS reads
// are in flight together): the first probe is the guess nearest to the
// lane's position tb in its hash bin, whose two energies say whether the
// interval is the guess or a neighbour; the interval's energies and cross
// sections are then read at that index.  Nearly every lane is done there;
// the rest walk (behind wave-uniform tests, one for all N, so the common
// case runs without lane masks).
template <int N>
__device__ __forceinline__ void window_search(const WinQ (&w)[N], float tb, double e, WinHit (&h)[N])
{
    uint32_t k[N];
    bool rare[N], glob[N];
    double eg[N], eg1[N];
#pragma unroll
    for (int n = 0; n < N; ++n) {
        // (bracket_guess in one fused multiply-add: a window holds at most
        // 64 points, so hi - lo is exact in float and the guess stays <= hi;
        // any guess in the bracket ends at the same interval)
        const uint32_t j = w[n].lo + (uint32_t)__builtin_fmaf(tb, (float)(w[n].hi - w[n].lo), 0.5f);
        const double *Ej = w[n].Ew + (int32_t)(j - w[n].wlo);
        eg[n] = Ej[0];
        eg1[n] = Ej[1];
        k[n] = j;
    }
    bool any_rare = false;
#pragma unroll
    for (int n = 0; n < N; ++n) {
        // (bitwise, not short-circuit, so that no load or compare waits
        // behind a branch)
        const uint32_t j = k[n];
        const bool dn = (j > w[n].lo) & (e < eg[n]);
        const bool up = !dn & (j < w[n].hi) & (e >= eg1[n]);
        k[n] = j + (up ? 1u : 0u) - (dn ? 1u : 0u);
        const uint32_t t = k[n] - w[n].wlo;
        h[n].e0 = w[n].Ew[t];
        h[n].e1 = w[n].Ew[t + 1u];
        h[n].x0 = w[n].Xw[t];
        h[n].x1 = w[n].Xw[t + 1u];
    }
#pragma unroll
    for (int n = 0; n < N; ++n) {
        // (at the grid's ends, k = 0 or k = len - 2, E outside [e0, e1) is
        // the clamped interval itself: the walks below then leave it as is)
        rare[n] = (e < h[n].e0) | (e >= h[n].e1);
        glob[n] = false;
        any_rare = any_rare || rare[n];
    }
    if (__ballot(any_rare)) {
#pragma unroll
        for (int n = 0; n < N; ++n) {
            if (rare[n]) {
                uint32_t kk = k[n];
                double e0 = h[n].e0, e1 = h[n].e1;
                while (kk > w[n].lo && e < e0) {
                    --kk;
                    e1 = e0;
                    e0 = w[n].Ew[kk - w[n].wlo];
                }
                while (kk < w[n].hi && e >= e1) {
                    ++kk;
                    e0 = e1;
                    e1 = w[n].Ew[kk + 1u - w[n].wlo];
                }
                glob[n] = (e < e0 && kk > 0u) || (e >= e1 && kk + 2u < w[n].len);
                k[n] = kk;
                h[n].e0 = e0;
                h[n].e1 = e1;
                h[n].x0 = w[n].Xw[kk - w[n].wlo];
                h[n].x1 = w[n].Xw[kk + 1u - w[n].wlo];
            }
        }
    }
    // k lies in the bracket, inside the window, and the cross sections came
    // from LDS; a lane whose hash bin was computed one off then walks to the
    // defined index in global memory and reloads
    bool any_glob = false;
#pragma unroll
    for (int n = 0; n < N; ++n) any_glob = any_glob || glob[n];
    if (__ballot(any_glob)) {
#pragma unroll
        for (int n = 0; n < N; ++n) {
            if (glob[n]) {
                uint32_t kk = k[n];
                const double *g = w[n].g;
                while (kk > 0u && e < g[kk]) --kk;
                while (kk + 2u < w[n].len && e >= g[kk + 1u]) ++kk;
                h[n].e0 = g[kk];
                h[n].e1 = g[kk + 1u];
                h[n].x0 = w[n].x[kk];
                h[n].x1 = w[n].x[kk + 1u];
            }
        }
        // these loads complete here (vmcnt 0), so that the common path,
        // which joins below, waits on none of them, and so not on the next
        // windows' loads issued before them either
        __builtin_amdgcn_s_waitcnt(0x0F70);
    }
}

// One nuclide on its own (the odd last one, or one of a pair whose windows do
// not fit half a wave each): its window loaded now into E_w / X_w when it
// holds at most WIN_PTS points, else a search of global memory.  Returns the
// micro cross sections in c, sg.
__device__ __forceinline__ void window_single(const XsDev &xs, const MatNuc &mn, uint32_t wlo, uint32_t wn,
                                              uint2 br, float tb, double e, double *E_w, double2 *X_w,
                                              uint32_t lane, double &c, double &sg)
{
    const double *g = xs.Eg + mn.off;
    const double2 *x = xs.xs + mn.off;
    double e0, e1;
    double2 x0, x1;
    if (wn <= (uint32_t)WIN_PTS) {
        double pe = 0.0;
        double2 px = make_double2(0.0, 0.0);
        if (lane < wn) {
            pe = g[wlo + lane];
            px = x[wlo + lane];
        }
        E_w[lane] = pe;
        X_w[lane] = px;
        wave_lds_sync();
        const WinQ w[1] = {{E_w, X_w, wlo, br.x, br.y, mn.len, g, x}};
        WinHit hit[1];
        window_search(w, tb, e, hit);
        e0 = hit[0].e0;
        e1 = hit[0].e1;
        x0 = hit[0].x0;
        x1 = hit[0].x1;
        wave_lds_sync();
    } else {
        const uint32_t k = grid_find(g, mn.len, br.x, br.y, e);
        e0 = g[k];
        e1 = g[k + 1u];
        x0 = x[k];
        x1 = x[k + 1u];
    }
    const double f = (e - e0) / (e1 - e0);
    c = x0.x + f * (x1.x - x0.x);
    sg = x0.y + f * (x1.y - x0.y);
}

// The interval fraction (E - E_i) / (E_(i+1) - E_i), correctly rounded, in
// the form the division's own instruction sequence takes when neither
// operand needs the scaling that sequence applies near the ends of the
// exponent range: the reciprocal refined by two Newton steps, the quotient
// and one fused correction (Markstein's theorem: correctly rounded).  With
// every grid energy and E in [2^-100, 2^100] the difference and the spacing
// lie in [2^-152, 2^101] (or the difference is 0), nothing is scaled and the
// special-case fix-up returns the quotient unchanged, so this is the same
// value as the division, in three instructions fewer.
__device__ __forceinline__ double frac_div(double n, double d)
{
    double r = __builtin_amdgcn_rcp(d);
    r = __builtin_fma(r, __builtin_fma(-d, r, 1.0), r);
    r = __builtin_fma(r, __builtin_fma(-d, r, 1.0), r);
    const double q = n * r;
    return __builtin_fma(__builtin_fma(-d, q, n), r, q);
}

// frac_div may serve the wave: the tables' energies lie in its range (a
// flag set with the tables) and so do the energies of all the wave's lanes.
__device__ __forceinline__ bool frac_div_wave(const LookupArgs &a, uint32_t i, bool valid)
{
    if (!a.xs.div_safe) return false;
    bool in = true;
    if (valid) {
        const double e = a.E[a.list ? a.list[i] : i];
        in = e >= 0x1p-100 && e <= 0x1p100;
    }
    return __ballot(!in) == 0;
}

// window_lookups without reaction channels, two nuclides at a time: when the
// windows of nuclides q and q + 1 hold at most half a wave's points each (all
// but ~1e-4 of the pairs of the 300-nuclide tables), one load per lane brings
// both (lanes 0-31 nuclide q's window, lanes 32-63 the other's), one LDS
// store and one wave sync stage them, and the two searches run side by side;
// the next pair's windows are loaded meanwhile.  A pair that does not fit,
// and an odd last nuclide, go one at a time.  The same intervals,
// interpolation, sums in material order and checkpoints as window_lookups:
// the results bit for bit.
template <bool FAST_DIV>
__device__ __forceinline__ int32_t window_lookups_pairs(const LookupArgs &a, const uint2 *sh, const int32_t *s_info,
                                                        uint32_t i, bool valid, double *we, double2 *wx)
{
    constexpr uint32_t HALF = WIN_PTS / 2;
    const XsDev &xs = a.xs;
    const uint64_t vmask = __ballot(valid);
    if (!vmask) return 0;
    const int32_t m = __builtin_amdgcn_readfirstlane(s_info[1]);
    const int32_t b0 = __builtin_amdgcn_readfirstlane(s_info[2]);
    const int32_t q0 = __builtin_amdgcn_readfirstlane(xs.mat_off[m]);
    const int32_t nk = __builtin_amdgcn_readfirstlane(xs.mat_off[m + 1]) - q0;
    // a lane past the end of the queue works on the wave's first particle
    // (same values, never stored), so the nuclide loop needs no lane mask
    const uint32_t i_own = valid ? i : i - (uint32_t)lane_id() + (uint32_t)(__ffsll((long long)vmask) - 1);
    const uint32_t p = a.list ? a.list[i_own] : i_own;
    const double e = a.E[p];
    const int32_t b = (int32_t)(a.keys[i_own] % (uint32_t)xs.M);
    const int32_t bmin = __builtin_amdgcn_readfirstlane(__shfl(b, __ffsll((long long)vmask) - 1, 64));
    const int32_t bmax = __builtin_amdgcn_readfirstlane(__shfl(b, 63 - __clzll((long long)vmask), 64));
    const uint2 *hmin = sh + (bmin - b0) * nk, *hmax = sh + (bmax - b0) * nk, *hown = sh + (b - b0) * nk;
    const uint32_t lane = (uint32_t)lane_id();
    double *E_w = we + 1 + (threadIdx.x & ~63u);  // one pad point before and after the waves' rows
    double2 *X_w = wx + (threadIdx.x & ~63u);
    const float tb = bin_position(xs, e, b);
    const int32_t cp_sh = a.cp && nk > CP_MIN_NUC ? cp_shift(nk) : 30;  // 30: never a checkpoint
    const int32_t cp_mask = (1 << cp_sh) - 1;
    CpPairs cpw{a.cp ? a.cp + (size_t)p * CP_MAX : nullptr, 0.0};
    double sa = 0.0, ss = 0.0;
    // the pair starting at nuclide q: its rows, windows (first point and
    // count, wave-uniform) and this lane's point, loaded one pair ahead
    struct Pair {
        MatNuc ma, mb;
        uint32_t wla, wna, wlb, wnb;
        bool fits;
    };
    auto load_pair = [&](int32_t q, Pair &r, double &pe, double2 &px) {
        r.ma = uniform_load(xs.mnuc, (int64_t)q0 + q);
        r.mb = uniform_load(xs.mnuc, (int64_t)q0 + q + 1);
        r.wla = __builtin_amdgcn_readfirstlane(hmin[q].x);
        r.wna = __builtin_amdgcn_readfirstlane(hmax[q].y) + 2u - r.wla;
        r.wlb = __builtin_amdgcn_readfirstlane(hmin[q + 1].x);
        r.wnb = __builtin_amdgcn_readfirstlane(hmax[q + 1].y) + 2u - r.wlb;
        r.fits = r.wna <= HALF && r.wnb <= HALF;
        pe = 0.0;
        px = make_double2(0.0, 0.0);
        if (r.fits) {
            const bool lo_half = lane < HALF;
            const uint32_t t = lo_half ? lane : lane - HALF;
            if (t < (lo_half ? r.wna : r.wnb)) {
                const uint32_t pt = lo_half ? r.ma.off + r.wla + t : r.mb.off + r.wlb + t;
                pe = xs.Eg[pt];
                px = xs.xs[pt];
            }
        }
    };
    auto accumulate = [&](int32_t q, const MatNuc &mn, double c, double sg) {
        sa = sa + mn.dens * c;
        ss = ss + mn.dens * sg;
        // (a lane past the queue's end writes the same values as the lane
        // whose particle it repeats, into that particle's row)
        const int32_t done = q + 1;
        if ((done & cp_mask) == 0) cpw.put((done >> cp_sh) - 1, ss);
    };
    Pair nxt{};
    double pe = 0.0;
    double2 px = make_double2(0.0, 0.0);
    if (nk >= 2) load_pair(0, nxt, pe, px);
    int32_t q = 0;
    for (; q + 1 < nk; q += 2) {
        const Pair cur = nxt;
        const double ce = pe;
        const double2 cx = px;
        if (q + 3 < nk) load_pair(q + 2, nxt, pe, px);
        const uint2 bra = hown[q], brb = hown[q + 1];  // this lane's brackets of q, q + 1
        double ca, sga, cb, sgb;
        if (cur.fits) {
            E_w[lane] = ce;
            X_w[lane] = cx;
            wave_lds_sync();
            const WinQ w[2] = {{E_w, X_w, cur.wla, bra.x, bra.y, cur.ma.len, xs.Eg + cur.ma.off, xs.xs + cur.ma.off},
                               {E_w + HALF, X_w + HALF, cur.wlb, brb.x, brb.y, cur.mb.len, xs.Eg + cur.mb.off,
                                xs.xs + cur.mb.off}};
            WinHit hit[2];
            window_search(w, tb, e, hit);
            wave_lds_sync();
            const double fa = FAST_DIV ? frac_div(e - hit[0].e0, hit[0].e1 - hit[0].e0)
                                       : (e - hit[0].e0) / (hit[0].e1 - hit[0].e0);
            const double fb = FAST_DIV ? frac_div(e - hit[1].e0, hit[1].e1 - hit[1].e0)
                                       : (e - hit[1].e0) / (hit[1].e1 - hit[1].e0);
            ca = hit[0].x0.x + fa * (hit[0].x1.x - hit[0].x0.x);
            sga = hit[0].x0.y + fa * (hit[0].x1.y - hit[0].x0.y);
            cb = hit[1].x0.x + fb * (hit[1].x1.x - hit[1].x0.x);
            sgb = hit[1].x0.y + fb * (hit[1].x1.y - hit[1].x0.y);
        } else {
            window_single(xs, cur.ma, cur.wla, cur.wna, bra, tb, e, E_w, X_w, lane, ca, sga);
            window_single(xs, cur.mb, cur.wlb, cur.wnb, brb, tb, e, E_w, X_w, lane, cb, sgb);
        }
        accumulate(q, cur.ma, ca, sga);
        accumulate(q + 1, cur.mb, cb, sgb);
    }
    if (q < nk) {  // the odd last nuclide
        const MatNuc mn = uniform_load(xs.mnuc, (int64_t)q0 + q);
        const uint32_t wlo = __builtin_amdgcn_readfirstlane(hmin[q].x);
        const uint32_t wn = __builtin_amdgcn_readfirstlane(hmax[q].y) + 2u - wlo;
        double c, sg;
        window_single(xs, mn, wlo, wn, hown[q], tb, e, E_w, X_w, lane, c, sg);
        accumulate(q, mn, c, sg);
    }
    if (!valid) return 0;
    if (cp_sh != 30) cpw.finish(nk >> cp_sh);
    if (a.Sa) a.Sa[p] = sa;
    if (a.Ss) a.Ss[p] = ss;
    if (a.flags) a.flags[p] = F_ALIVE;
    return nk;
}

// DIAG: the per-nuclide outputs (idx_out, sc_out, ss_out) may be set; the
// transport's lookups run without them, in fewer registers.  CHAN: the
// reaction channels are assembled in the same pass (same index and fraction
// per nuclide) into sx.
// WIN: sorted queues take window_lookups in staged workgroups.
template <int ILP, bool DIAG, bool CHAN, bool WIN = false>
__global__ void __launch_bounds__(WG) k_lookup(LookupArgs a)
{
    __shared__ uint2 sh[LDS_HASH_PAIRS];
    __shared__ int32_t s_info[4];
    __shared__ double s_we[WIN ? WG + 2 : 1];
    __shared__ double2 s_wx[WIN ? WG : 1];
    __shared__ double s_wc[(WIN && CHAN) ? WAVES * WIN_CHAN : 1];
    const XsDev &xs = a.xs;
    const uint32_t n = a.n_ptr ? *a.n_ptr : a.n_fixed;
    // a sorted queue: runs of XCD_CHUNK neighbouring blocks on one XCD, so
    // that workgroups sharing hash bins (and so grid windows) share one L2
    const uint32_t blk = a.keys ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x;
    const uint32_t i0 = blk * WG;
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
                nrow = (int32_t)(k1 % (uint32_t)xs.M) - b0 + 1;
                if (nrow * nk <= LDS_HASH_PAIRS) { staged = 1; m = m0; }
            }
        }
        s_info[0] = staged; s_info[1] = m; s_info[2] = b0; s_info[3] = nrow;
    }
    __syncthreads();
    const bool staged = s_info[0] != 0;
    if (staged) {
        const int32_t m = s_info[1], b0 = s_info[2], nrow = s_info[3];
        const int32_t nk = xs.mat_off[m + 1] - xs.mat_off[m];
        const uint2 *src = hash_row(xs, m, b0, nk);
        for (int32_t t = threadIdx.x; t < nrow * nk; t += WG) sh[t] = src[t];
        __syncthreads();
    }
    int32_t nk_done = 0;
    if (WIN && staged) {
        if constexpr (CHAN) nk_done = window_lookups<CHAN>(a, sh, s_info, i, valid, s_we, s_wx, s_wc);
        else if (frac_div_wave(a, i, valid))
            nk_done = window_lookups_pairs<true>(a, sh, s_info, i, valid, s_we, s_wx);
        else
            nk_done = window_lookups_pairs<false>(a, sh, s_info, i, valid, s_we, s_wx);
    } else if (valid) {
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
        if (CHAN)
            for (int32_t x = 0; x < xs.n_chan; ++x) a.sx[(size_t)p * xs.n_chan + x] = NAN;
        m = -1;
    }
    if (m >= 0) {
    const int32_t q0 = xs.mat_off[m];
    const int32_t nk = xs.mat_off[m + 1] - q0;
    const float tb = bin_position(xs, e, b);
    double sa = 0.0, ss = 0.0;
    const MatNuc *mnuc = xs.mnuc + q0;
    const int32_t cp_sh = a.cp && nk > CP_MIN_NUC ? cp_shift(nk) : 30;  // 30: never a checkpoint
    const int32_t cp_mask = (1 << cp_sh) - 1;
    CpPairs cpw{a.cp ? a.cp + (size_t)p * CP_MAX : nullptr, 0.0};
    double acc[MAX_CHAN];
    if (CHAN) {
#pragma unroll
        for (int x = 0; x < MAX_CHAN; ++x) acc[x] = 0.0;
    }
    // the nuclide loop, once with the brackets in LDS and once in global memory
    auto nuclides = [&](const uint2 *h0) {
        for (int32_t q = 0; q < nk; q += ILP) {
            const int32_t cnt = nk - q < ILP ? nk - q : ILP;
            double dens[ILP], c[ILP], s[ILP], fr[ILP];
            uint32_t ix[ILP], pt[ILP];
            micro_group<ILP>(xs, mnuc, h0, nk, q, cnt, e, tb, dens, ix, c, s, fr, pt);
            if (CHAN) channel_group<ILP>(xs, cnt, dens, fr, pt, acc);
            // the sum runs in material order, one nuclide after the other
#pragma unroll
            for (int k = 0; k < ILP; ++k) {
                if (k < cnt) {
                    sa = sa + dens[k] * c[k];
                    ss = ss + dens[k] * s[k];
                    const int32_t done = q + k + 1;  // a checkpoint of the scattering sum
                    if ((done & cp_mask) == 0) cpw.put((done >> cp_sh) - 1, ss);
                    if (DIAG) {
                        if (a.idx_out) a.idx_out[(size_t)p * nk + q + k] = (int32_t)ix[k];
                        if (a.sc_out) a.sc_out[(size_t)p * nk + q + k] = c[k];
                        if (a.ss_out) a.ss_out[(size_t)p * nk + q + k] = s[k];
                    }
                }
            }
        }
    };
    if (staged) nuclides(sh + (b - s_info[2]) * nk);
    else nuclides(hash_row(xs, m, b, nk));
    if (cp_sh != 30) cpw.finish(nk >> cp_sh);
    if (a.Sa) a.Sa[p] = sa;
    if (a.Ss) a.Ss[p] = ss;
    if (CHAN) {
#pragma unroll
        for (int x = 0; x < MAX_CHAN; ++x)
            if (x < xs.n_chan) a.sx[(size_t)p * xs.n_chan + x] = acc[x];
    }
    if (a.flags) a.flags[p] = F_ALIVE;
    nk_done = nk;
    }
    }
    if (a.nuc_count) {
        const uint32_t c = wave_sum_u32((uint32_t)nk_done);
        if (lane_id() == 0 && c) atomicAdd(a.nuc_count, (unsigned long long)c);
    }
}

// Lookup on the unionized grid of the particle's material: one search in the
// union grid (hash bracket, bisection, walk), then each nuclide's interval is
// read from the union point's index row instead of searched.  Same intervals,
// same interpolation and sums in material order as k_lookup, so the same
// results bit for bit (scattering-sum checkpoints included).
template <int ILP>
__global__ void __launch_bounds__(WG) k_lookup_union(LookupArgs a)
{
    const XsDev &xs = a.xs;
    const uint32_t n = a.n_ptr ? *a.n_ptr : a.n_fixed;
    const uint32_t i = blockIdx.x * WG + threadIdx.x;
    int32_t nk_done = 0;
    if (i < n) {
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
        if (m < 0 || m >= xs.n_mat) {
            if (a.Sa) a.Sa[p] = NAN;
            if (a.Ss) a.Ss[p] = NAN;
        } else {
            const UnionMat um = xs.um[m];
            const double *U = xs.ug + um.g_off;
            const uint32_t last = um.n - 1u;
            uint32_t lo = xs.uh[um.h_off + b], hi = xs.uh[um.h_off + b + 1] + 1u;
            hi = hi < last ? hi : last;
            lo = lo < hi ? lo : hi;
            while (lo < hi) {  // largest u in [lo, hi] with U_u <= E
                const uint32_t mid = (lo + hi + 1u) >> 1;
                if (U[mid] <= e) lo = mid; else hi = mid - 1u;
            }
            uint32_t u = lo;  // a bin computed one off: walk to the defined point
            while (u > 0u && e < U[u]) --u;
            while (u < last && e >= U[u + 1u]) ++u;
            const int32_t q0 = xs.mat_off[m];
            const int32_t nk = xs.mat_off[m + 1] - q0;
            const uint32_t *row = xs.ui + um.i_off + (uint64_t)u * (uint64_t)nk;
            const MatNuc *mnuc = xs.mnuc + q0;
            const int32_t cp_sh = a.cp && nk > CP_MIN_NUC ? cp_shift(nk) : 30;
            const int32_t cp_mask = (1 << cp_sh) - 1;
            CpPairs cpw{a.cp ? a.cp + (size_t)p * CP_MAX : nullptr, 0.0};
            double sa = 0.0, ss = 0.0;
            for (int32_t q = 0; q < nk; q += ILP) {
                const int32_t cnt = nk - q < ILP ? nk - q : ILP;
                double dens[ILP], e0[ILP], e1[ILP];
                double2 x0[ILP], x1[ILP];
#pragma unroll
                for (int k = 0; k < ILP; ++k) {
                    const int32_t qk = q + (k < cnt ? k : 0);
                    const MatNuc mn = mnuc[qk];
                    const uint32_t pt = mn.off + row[qk];
                    dens[k] = mn.dens;
                    e0[k] = xs.Eg[pt];
                    e1[k] = xs.Eg[pt + 1u];
                    x0[k] = xs.xs[pt];
                    x1[k] = xs.xs[pt + 1u];
                }
#pragma unroll
                for (int k = 0; k < ILP; ++k) {
                    if (k < cnt) {
                        const double f = (e - e0[k]) / (e1[k] - e0[k]);
                        const double c = x0[k].x + f * (x1[k].x - x0[k].x);
                        const double s = x0[k].y + f * (x1[k].y - x0[k].y);
                        sa = sa + dens[k] * c;
                        ss = ss + dens[k] * s;
                        const int32_t done = q + k + 1;
                        if ((done & cp_mask) == 0) cpw.put((done >> cp_sh) - 1, ss);
                    }
                }
            }
            if (cp_sh != 30) cpw.finish(nk >> cp_sh);
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

// Windowed-multipole macroscopic cross sections: per nuclide of the
// material, u = sqrt(E), the window holding u, its poles' terms
// Re[r sqrt(pi) beta w(beta (u - p))] / E and the background polynomial in u;
// sums in material order.  pole_count (nullable) adds the poles evaluated.
__global__ void __launch_bounds__(WG) k_lookup_mp(MpDev mp, uint32_t n, const double *E, const int32_t *mat,
                                                  double *Sa, double *Ss, unsigned long long *pole_count)
{
    const uint32_t i = blockIdx.x * WG + threadIdx.x;
    uint32_t poles = 0;
    if (i < n) {
        const double e = E[i];
        const int32_t m = mat[i];
        if (m < 0 || m >= mp.n_mat) {
            Sa[i] = NAN;
            Ss[i] = NAN;
        } else {
            const double u = sqrt(e);
            const double spi = 1.7724538509055160273;  // sqrt(pi)
            double sa = 0.0, ss = 0.0;
            for (int32_t q = mp.mat_off[m]; q < mp.mat_off[m + 1]; ++q) {
                const MpNuc nd = mp.nuc[mp.mat_nuc[q]];
                const double beta = mp.mat_beta[q];
                int32_t w = (int32_t)floor((u - nd.u_lo) / nd.du);
                w = w < 0 ? 0 : (w > nd.n_windows - 1 ? nd.n_windows - 1 : w);
                const int2 rg = mp.win[nd.w_off + w];
                const double spb = spi * beta;
                double c = 0.0, s = 0.0;
                for (int32_t j = rg.x; j < rg.y; ++j) {
                    const double2 p = mp.poles[nd.p_off + j];
                    double wr, wi;
                    faddeeva(mp, beta * (u - p.x), -beta * p.y, wr, wi);
                    const double cr = spb * wr, ci = spb * wi;
                    const double2 a = mp.rc[nd.p_off + j], b = mp.rs[nd.p_off + j];
                    c += a.x * cr - a.y * ci;
                    s += b.x * cr - b.y * ci;
                }
                poles += (uint32_t)(rg.y - rg.x);
                c = c / e;
                s = s / e;
                double up = 1.0 / u;
                const double *bc = mp.bgc + nd.bg_off + (size_t)w * nd.n_bg;
                const double *bs = mp.bgs + nd.bg_off + (size_t)w * nd.n_bg;
                for (int32_t k = 0; k < nd.n_bg; ++k) {
                    c += bc[k] * up;
                    s += bs[k] * up;
                    up *= u;
                }
                sa = sa + mp.mat_dens[q] * c;
                ss = ss + mp.mat_dens[q] * s;
            }
            Sa[i] = sa;
            Ss[i] = ss;
        }
    }
    if (pole_count) {
        const uint32_t t = wave_sum_u32(poles);
        if (lane_id() == 0 && t) atomicAdd(pole_count, (unsigned long long)t);
    }
}

// ---------------------------------------------------------------------------
// advance: sample the flight, move, score track length
// ---------------------------------------------------------------------------
template <int WWK>
__device__ __forceinline__ void end_copy(const BankDev &b, const WwDev &W, uint32_t s, Particle &p, int32_t fate,
                                         HistLog *log, uint64_t first_pid);

// Flight of every alive particle.  CROSS (analog runs without an importance
// grid): a particle whose flight ends on a surface crosses it here, from the
// state the flight has in registers, instead of in k_cross (one pass over the
// bank fewer); it is marked EV_DONE, and the split queues only collisions.
// A particle at the event cap then ends here as lost too.
// LOG: the history log may be on; without it (the transport's runs) the
// fields only the log reads are never loaded or kept, in fewer registers.
template <bool CROSS, bool LOG>
__global__ void __launch_bounds__(WG) k_advance(BankDev b, GeomDev g, TallyDev tal, WwDev W, const Counters *ctr,
                                                uint64_t seed, int64_t max_events, int32_t log_on, HistLog *log,
                                                uint64_t first_pid, unsigned long long *lost)
{
    if constexpr (!LOG) {
        log = nullptr;
        log_on = 0;
    }
    extern __shared__ double slab[];
    __shared__ double gl[N_GLOBAL * WAVES];
    const uint32_t n = ctr->nA;
    const uint32_t i0 = blockIdx.x * WG;
    if (i0 >= n) return;
    const uint32_t i = i0 + threadIdx.x;
    StepScore sc;
    clear_score(sc);
    int32_t flight_mat = -1;              // material of this lane's flight (-1: none)
    const double *sx_row = b.sx;
    // a mesh tally scores last, after the crossing, the stores and the
    // workgroup's tally rows: on gfx950 a load waits for every earlier
    // store and atomic of its wave, so no load may follow the mesh's atomic
    // adds; the flight's start, direction, length and weight wait here
    const bool mesh = tal.enabled && g.tally_kind == TALLY_MESH;
    bool mesh_on = false;
    double fx = 0.0, fy = 0.0, fz = 0.0, fu = 0.0, fv = 0.0, fw = 0.0, fd = 0.0, fwt = 0.0;
    if (i < n) {
        const uint32_t s = n == b.C ? i : b.A[i];  // every slot alive: the queue is the identity
        if ((int64_t)b.ncoll[s] + b.ncross[s] >= max_events) {
            if constexpr (CROSS) {  // event cap reached: the history ends here as lost
                Particle p = load_particle(b, s);
                atomicAdd(lost, 1ull);
                end_copy<WW_OFF>(b, W, s, p, FATE_LOST, log, first_pid);
                b.event[s] = EV_DONE;
            } else {
                b.event[s] = 0xFF;  // the cross kernel ends it as lost
            }
        } else {
            Particle p = load_particle(b, s);
            const double x0 = p.x;
            fx = p.x; fy = p.y; fz = p.z; fu = p.u; fv = p.v; fw = p.w; fwt = p.wt;
            flight_mat = p.mat;
            if (tal.chan) sx_row = b.sx + (size_t)s * tal.n_chan;
            fd = do_advance(p, g, seed, tal.enabled != 0, mesh ? nullptr : tal.mesh_tl, log_on != 0, sc);
            mesh_on = mesh;
            if (!CROSS && W.imp_nx) imp_enter(W, s, x0, p.x, p.E, p.wt);
            b.ndraw[s] = p.ndraw;
            if (log_on) b.track[s] = p.track;
            if (CROSS && p.ev != EV_COLLIDE) {
                bool need_lookup, leak_xhi;
                const int32_t fate = do_cross(p, g, sc, need_lookup, leak_xhi);
                b.ncross[s] = p.ncross;
                if (fate) {
                    end_copy<WW_OFF>(b, W, s, p, fate, log, first_pid);
                } else {
                    b.x[s] = p.x; b.y[s] = p.y; b.z[s] = p.z;
                    b.u[s] = p.u; b.v[s] = p.v; b.w[s] = p.w;
                    b.cell[s] = p.cell;
                    b.inside[s] = p.inside ? 1 : 0;
                    b.mat[s] = p.mat;
                    if (need_lookup) b.flags[s] = F_ALIVE | F_LOOKUP;
                }
                b.event[s] = EV_DONE;
            } else {
                b.x[s] = p.x; b.y[s] = p.y; b.z[s] = p.z;
                b.event[s] = p.ev;
            }
        }
    }
    if (tal.enabled && g.tally_kind != TALLY_MESH)
        wg_bin_add(sc.tl_bin, sc.tl_val, slab, tal.n_bins, tal.tl + (size_t)blockIdx.x * tal.n_bins);
    if (tal.enabled && tal.chan)
        wg_chan_add(flight_mat, sc.g[G_TRACK], sx_row, tal.n_chan, slab, tal.chan_bins,
                    tal.chan + (size_t)blockIdx.x * tal.chan_bins);
    wg_glob_add(sc.g, gl, tal.glob + (size_t)blockIdx.x * N_GLOBAL);
    if (mesh_on) mesh_flight(g, tal.mesh_tl, fx, fy, fz, fu, fv, fw, fd, fwt);
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
                const uint8_t ev = b.event[n == b.C ? i : b.A[i]];
                cc += ev == EV_COLLIDE ? 1u : 0u;
                cx += ev != EV_COLLIDE && ev != EV_DONE ? 1u : 0u;
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
    // every item's slot and event loaded before any queue entry is stored (a
    // load waits for the earlier stores of its wave)
    uint32_t sl[TILE_ITEMS];
    uint8_t evs[TILE_ITEMS];
#pragma unroll
    for (int r = 0; r < TILE_ITEMS; ++r) {
        const uint32_t i = base + r * WG + threadIdx.x;
        sl[r] = i < n ? (n == b.C ? i : b.A[i]) : 0u;
    }
#pragma unroll
    for (int r = 0; r < TILE_ITEMS; ++r) evs[r] = base + r * WG + threadIdx.x < n ? b.event[sl[r]] : 0;
    for (int r = 0; r < TILE_ITEMS; ++r) {
        const uint32_t i = base + r * WG + threadIdx.x;
        const bool valid = i < n;
        const uint32_t s = sl[r];
        const uint8_t ev = evs[r];
        const bool pc = valid && ev == EV_COLLIDE;
        const bool px = valid && ev != EV_COLLIDE && ev != EV_DONE;
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
// end of a copy, and the state a step leaves in the bank
// ---------------------------------------------------------------------------
// The copy in slot s died with `fate`: the next pending copy of its history
// takes the slot (alive, lookup due), or the history ends (slot free).
template <int WWK>
__device__ __forceinline__ void end_copy(const BankDev &b, const WwDev &W, uint32_t s, Particle &p, int32_t fate,
                                         HistLog *log, uint64_t first_pid)
{
    if constexpr (WWK != WW_OFF) {
        if (log) log_copy(log, first_pid, p, fate, W, s);
        if (ww_pending(W, s)) {
            ww_pop(W, s, p);
            b.x[s] = p.x; b.y[s] = p.y; b.z[s] = p.z;
            b.u[s] = p.u; b.v[s] = p.v; b.w[s] = p.w;
            b.E[s] = p.E; b.wt[s] = p.wt;
            b.cell[s] = p.cell; b.mat[s] = p.mat; b.inside[s] = p.inside ? 1 : 0;
            b.ncoll[s] = p.ncoll; b.ncross[s] = p.ncross;
            b.lineage[s] = p.lineage; b.ndraw[s] = p.ndraw;
            b.track[s] = p.track;
            b.flags[s] = F_ALIVE | F_LOOKUP;
        } else {
            b.flags[s] = 0;
        }
    } else {
        b.flags[s] = 0;
        if (log) write_log(log, first_pid, p, fate);
    }
}

// ---------------------------------------------------------------------------
// surface crossing
// ---------------------------------------------------------------------------
template <int WWK>
__global__ void __launch_bounds__(WG) k_cross(BankDev b, GeomDev g, TallyDev tal, WwDev W, const Counters *ctr,
                                              uint64_t seed, HistLog *log, uint64_t first_pid,
                                              unsigned long long *lost)
{
    __shared__ double gl[N_GLOBAL * WAVES];
    const uint32_t n = ctr->nX;
    const uint32_t i0 = blockIdx.x * WG;
    if (i0 >= n) return;
    const uint32_t i = i0 + threadIdx.x;
    const bool act = i < n;
    StepScore sc;
    clear_score(sc);
    Particle p{};
    uint32_t s = 0;
    int32_t fate = 0;
    bool need_lookup = false;
    if (act) {
        s = b.Qx[i];
        p = load_particle(b, s);
        if (p.ev == 0xFF) {
            fate = FATE_LOST;
            atomicAdd(lost, 1ull);
        } else {
            bool leak_xhi;
            fate = do_cross(p, g, sc, need_lookup, leak_xhi);
            if (leak_xhi && W.imp_nx) imp_credit(W, s, p.wt);
        }
    }
    if constexpr (WWK != WW_OFF) {
        const bool chk = act && fate == 0;
        const double ln_i = ww_ln_importance<WWK>(W, p, chk);
        if (chk) fate = ww_check(W, s, p, ln_i, seed, sc);
    }
    if (act) {
        b.ncross[s] = p.ncross;
        if (fate) {
            end_copy<WWK>(b, W, s, p, fate, log, first_pid);
        } else {
            b.x[s] = p.x; b.y[s] = p.y; b.z[s] = p.z;
            b.u[s] = p.u; b.v[s] = p.v; b.w[s] = p.w;
            b.cell[s] = p.cell;
            b.inside[s] = p.inside ? 1 : 0;
            b.mat[s] = p.mat;
            if constexpr (WWK != WW_OFF) {
                b.wt[s] = p.wt;
                b.ndraw[s] = p.ndraw;
            }
            if (need_lookup) b.flags[s] = F_ALIVE | F_LOOKUP;
        }
    }
    wg_glob_add(sc.g, gl, tal.glob + (size_t)blockIdx.x * N_GLOBAL);
}

// ---------------------------------------------------------------------------
// collision: analog capture or elastic scattering off a target at rest
// ---------------------------------------------------------------------------
// `list` is the collide queue, in split order or sorted by (material, hash
// bin of E) so that the gathers of neighbouring lanes share cache lines.
template <int WWK, bool LOG>
__global__ void __launch_bounds__(WG) k_collide(BankDev b, const uint32_t *list, XsDev xs, GeomDev g, TallyDev tal,
                                                WwDev W, const Counters *ctr, uint64_t seed, HistLog *log,
                                                uint64_t first_pid)
{
    if constexpr (!LOG) log = nullptr;  // (as in k_advance)
    extern __shared__ double slab[];
    __shared__ double gl[N_GLOBAL * WAVES];
    const uint32_t n = ctr->nC;
    const uint32_t i0 = blockIdx.x * WG;
    if (i0 >= n) return;
    const uint32_t i = i0 + threadIdx.x;
    const bool act = i < n;
    StepScore sc;
    clear_score(sc);
    Particle p{};
    uint32_t s = 0;
    int32_t fate = 0;
    // the collision estimator's mesh cell scores last (no load may follow an
    // atomic add of the wave: it would wait for it)
    const bool mesh = tal.enabled && g.tally_kind == TALLY_MESH;
    int32_t mesh_cell = -1;
    double mesh_val = 0.0;
    if (act) {
        s = list[i];
        p = load_particle(b, s);
        if (mesh) {
            mesh_cell = mesh_index(g, p.x, p.y, p.z);
            mesh_val = p.wt / (p.Sa + p.Ss);
        }
        fate = do_collide(p, xs, g, seed, tal.enabled != 0, mesh ? nullptr : tal.mesh_coll, sc,
                          b.cp ? b.cp + (size_t)s * CP_MAX : nullptr);
        if (fate == 0 && W.imp_nx) imp_enter(W, s, p.x, p.x, p.E, p.wt);
    }
    if constexpr (WWK != WW_OFF) {
        const bool chk = act && fate == 0;
        const double ln_i = ww_ln_importance<WWK>(W, p, chk);
        if (chk) fate = ww_check(W, s, p, ln_i, seed, sc);
    }
    if (act) {
        b.ncoll[s] = p.ncoll;
        b.ndraw[s] = p.ndraw;
        if (fate) {
            end_copy<WWK>(b, W, s, p, fate, log, first_pid);
        } else {
            b.E[s] = p.E;
            b.u[s] = p.u; b.v[s] = p.v; b.w[s] = p.w;
            if constexpr (WWK != WW_OFF) b.wt[s] = p.wt;
            b.flags[s] = F_ALIVE | F_LOOKUP;
        }
    }
    if (tal.enabled && g.tally_kind != TALLY_MESH)
        wg_bin_add(sc.c_bin, sc.c_val, slab, tal.n_bins, tal.coll + (size_t)blockIdx.x * tal.n_bins);
    wg_glob_add(sc.g, gl, tal.glob + (size_t)blockIdx.x * N_GLOBAL);
    if (mesh_cell >= 0) mesh_add(tal.mesh_coll, mesh_cell, mesh_val, g.n_bins);
}

// ---------------------------------------------------------------------------
// tile transport: each lane runs its particle to the end, the workgroup steps
// through lookup, flight and collision-or-crossing together so that the
// tallies are still added per step, in a fixed order, into the tile's rows
// ---------------------------------------------------------------------------
struct TileRows {
    double *tl, *coll, *glob;  // this tile's rows (tl/coll: n_bins doubles, glob: N_GLOBAL)
    double *mesh_tl, *mesh_coll;
    int32_t n_bins;
    bool enabled;              // binned flux tallies on
    double *chan;              // reaction-rate row (chan_bins doubles; the CHAN tiles)
    int32_t chan_bins, n_chan;
};

// ILP: nuclides per lane in lockstep in the lookup and the collision's walk
// (the tail runs few particles per compute unit: latency, not registers,
// bounds it, so it takes more).
// CHAN: the lookups also assemble the reaction channels into sx_row and the
// flights score their reaction rates.
template <int ILP, bool CHAN>
__device__ inline void run_tile(Particle &p, bool alive, bool need, const XsDev &xs, const GeomDev &g,
                                const TileRows &r, uint64_t seed, int64_t max_events, HistLog *log,
                                uint64_t log_first_pid, unsigned long long *lost, double *slab, double *gl,
                                double *sx_row, double *cp_row)
{
    const bool binned = r.enabled && g.tally_kind != TALLY_MESH;
    const bool log_on = log != nullptr;
    while (__syncthreads_or(alive)) {
        StepScore sc;
        clear_score(sc);
        int32_t fate = 0;
        if (alive && need) {
            do_lookup<ILP, CHAN>(p, xs, sx_row, cp_row);
            need = false;
        }
        int32_t flight_mat = -1;
        if (alive && (int64_t)p.ncoll + p.ncross >= max_events) {
            fate = FATE_LOST;
            atomicAdd(lost, 1ull);
        } else if (alive) {
            flight_mat = p.mat;
            do_advance(p, g, seed, r.enabled, r.mesh_tl, log_on, sc);
        }
        if (binned) wg_bin_add(sc.tl_bin, sc.tl_val, slab, r.n_bins, r.tl);
        if (CHAN && r.enabled) wg_chan_add(flight_mat, sc.g[G_TRACK], sx_row, r.n_chan, slab, r.chan_bins, r.chan);
        if (alive && fate == 0) {
            if (p.ev == EV_COLLIDE) {
                fate = do_collide<ILP>(p, xs, g, seed, r.enabled, r.mesh_coll, sc, cp_row);
                need = fate == 0;
            } else {
                bool leak_xhi;
                fate = do_cross(p, g, sc, need, leak_xhi);
            }
        }
        if (binned) wg_bin_add(sc.c_bin, sc.c_val, slab, r.n_bins, r.coll);
        wg_glob_add(sc.g, gl, r.glob);
        if (alive && fate != 0) {
            alive = false;
            if (log) write_log(log, log_first_pid, p, fate);
        }
    }
}

constexpr int TAIL_ILP = 4;

// Tail: when no history remains to start and few particles are in flight,
// one launch finishes them (workgroup row = blockIdx.x); the histories are
// the ones the event kernels would give.  Analog transport only: with weight
// windows a history's copies run in parallel in the event kernels.
template <bool CHAN>
__global__ void __launch_bounds__(WG) k_tail(BankDev b, XsDev xs, GeomDev g, TallyDev tal, const Counters *ctr,
                                             uint64_t seed, int64_t max_events, HistLog *log, uint64_t first_pid,
                                             unsigned long long *lost)
{
    extern __shared__ double slab[];
    __shared__ double gl[N_GLOBAL * WAVES];
    const uint32_t n = ctr->nA;
    const uint32_t i0 = blockIdx.x * WG;
    if (i0 >= n) return;
    const uint32_t i = i0 + threadIdx.x;
    Particle p{};
    uint32_t s = 0;
    bool alive = false, need = false;
    if (i < n) {
        s = b.A[i];
        p = load_particle(b, s);
        alive = true;
        need = (b.flags[s] & F_LOOKUP) != 0;
    }
    TileRows r;
    r.tl = tal.tl + (size_t)blockIdx.x * tal.n_bins;
    r.coll = tal.coll + (size_t)blockIdx.x * tal.n_bins;
    r.glob = tal.glob + (size_t)blockIdx.x * N_GLOBAL;
    r.mesh_tl = tal.mesh_tl;
    r.mesh_coll = tal.mesh_coll;
    r.n_bins = tal.n_bins;
    r.enabled = tal.enabled != 0;
    r.chan = CHAN ? tal.chan + (size_t)blockIdx.x * tal.chan_bins : nullptr;
    r.chan_bins = tal.chan_bins;
    r.n_chan = tal.n_chan;
    double *sx_row = CHAN ? b.sx + (size_t)s * tal.n_chan : nullptr;
    // the slot's checkpoint row: written by the lookups of the event loop and
    // of this kernel, read by the collisions of both
    double *cp_row = b.cp ? b.cp + (size_t)s * CP_MAX : nullptr;
    run_tile<TAIL_ILP, CHAN>(p, alive, need, xs, g, r, seed, max_events, log, first_pid, lost, slab, gl, sx_row,
                             cp_row);
    if (i < n) b.flags[s] = 0;
}

// ---------------------------------------------------------------------------
// problem set: many independent problems in one persistent launch
// ---------------------------------------------------------------------------
// Workgroups pull tiles (problem, range of its histories) from a queue until
// none is left.  Each tile writes only its own tally rows, so the per-problem
// sums, taken over the problem's tiles in tile order, do not depend on which
// workgroup ran which tile.
__device__ __forceinline__ void source_particle(Particle &p, const GeomDev &g, uint64_t pid, uint64_t seed)
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
    p.x = x; p.y = y; p.z = z;
    p.u = u; p.v = v; p.w = w;
    p.E = g.src_E;
    p.wt = 1.0;
    p.Sa = 0.0; p.Ss = 0.0; p.track = 0.0;
    p.pid = pid;
    p.ndraw = rng.n;
    p.lineage = 0u;
    p.cell = cell;
    p.inside = inside;
    p.mat = region_material(g, cell, inside);
    p.ncoll = 0;
    p.ncross = 0;
    p.ev = 0;
}

__global__ void __launch_bounds__(WG) k_problem_set(SetDev set, XsDev xs, int64_t max_events)
{
    extern __shared__ double slab[];
    __shared__ double gl[N_GLOBAL * WAVES];
    __shared__ uint32_t s_tile;
    const uint64_t batch = *set.batch;
    for (;;) {
        if (threadIdx.x == 0) s_tile = atomicAdd(set.next_tile, 1u);
        __syncthreads();
        const uint32_t t = s_tile;
        __syncthreads();
        if (t >= set.n_tiles) break;
        const SetTile tile = set.tiles[t];
        const SetProblem &P = set.problems[tile.problem];
        const uint64_t first_pid = P.pid_base + batch * P.histories;
        for (uint32_t r0 = 0; r0 < tile.count; r0 += WG) {
            Particle p{};
            const bool alive = r0 + threadIdx.x < tile.count;
            if (alive) source_particle(p, P.g, first_pid + tile.first + r0 + threadIdx.x, P.seed);
            TileRows r;
            r.tl = set.tl + (size_t)tile.row;
            r.coll = set.coll + (size_t)tile.row;
            r.glob = set.glob + (size_t)t * N_GLOBAL;
            r.mesh_tl = nullptr;
            r.mesh_coll = nullptr;
            r.n_bins = P.g.n_bins;
            r.enabled = true;
            r.chan = nullptr;
            r.chan_bins = r.n_chan = 0;
            HistLog *log = set.log ? set.log + P.log_off : nullptr;
            run_tile<DEFAULT_LOOKUP_ILP, false>(p, alive, true, xs, P.g, r, P.seed, max_events, log, first_pid,
                                                set.lost, slab, gl, nullptr, nullptr);
        }
    }
}

// Per-problem batch statistics: T = (sum of the problem's tile rows in tile
// order) / histories; S1 += T, S2 += T^2; then the batch counter advances.
// One workgroup per problem.
__global__ void __launch_bounds__(WG) k_problem_set_stats(SetDev set)
{
    const SetProblem &P = set.problems[blockIdx.x];
    const int32_t nb = P.g.n_bins;
    const double inv_n = 1.0 / (double)P.histories;
    for (int32_t k = threadIdx.x; k < 2 * nb + N_GLOBAL; k += WG) {
        double s = 0.0;
        for (uint32_t t = P.first_tile; t < P.first_tile + P.n_tiles; ++t) {
            const SetTile &tile = set.tiles[t];
            double v;
            if (k < nb) v = set.tl[tile.row + k];
            else if (k < 2 * nb) v = set.coll[tile.row + (k - nb)];
            else v = set.glob[(size_t)t * N_GLOBAL + (k - 2 * nb)];
            s = s + v;
        }
        const double T = s * inv_n;
        double *S1 = set.S1 + P.stat_off, *S2 = set.S2 + P.stat_off;
        S1[k] = S1[k] + T;
        S2[k] = S2[k] + T * T;
    }
}

__global__ void k_problem_set_next(SetDev set) { *set.batch = *set.batch + 1; }

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

// T = (sum of the partials in chunk order, or the fixed-point mesh
// accumulator `direct`) / n; S1 += T; S2 += T^2 (S2 == nullptr: S1 = T, the
// batch value alone).
__global__ void __launch_bounds__(WG) k_batch_stats(const double *partial, const double *direct,
                                                    int32_t n_cols, double inv_n, double *S1, double *S2)
{
    const int32_t k = blockIdx.x * WG + threadIdx.x;
    if (k >= n_cols) return;
    double s = 0.0;
    if (direct) {
        s = (double)reinterpret_cast<const unsigned long long *>(direct)[k] * MESH_FIX_INV;
    } else {
        for (int c = 0; c < RED_CHUNKS; ++c) s = s + partial[(size_t)c * n_cols + k];
    }
    const double T = s * inv_n;
    if (!S2) {
        S1[k] = T;
        return;
    }
    S1[k] = S1[k] + T;
    S2[k] = S2[k] + T * T;
}

// S1 += T_b, S2 += T_b^2 for the batch values T[b * stride + off + k],
// b = 0 .. n_b-1 in order (as n_b batch-statistics updates would).
__global__ void __launch_bounds__(WG) k_batch_accum(const double *T, int32_t n_b, int32_t stride, int32_t off,
                                                    int32_t n_cols, double *S1, double *S2)
{
    const int32_t k = blockIdx.x * WG + threadIdx.x;
    if (k >= n_cols) return;
    double s1 = S1[k], s2 = S2[k];
    for (int32_t b = 0; b < n_b; ++b) {
        const double t = T[(size_t)b * stride + off + k];
        s1 = s1 + t;
        s2 = s2 + t * t;
    }
    S1[k] = s1;
    S2[k] = s2;
}

// ---------------------------------------------------------------------------
// host-side launch wrappers
// ---------------------------------------------------------------------------
static inline unsigned blocks_for(size_t n, size_t per) { return (unsigned)((n + per - 1) / per); }

// LDS of the per-wave tally slabs (none when the binned tallies are off or
// use the mesh path)
// LDS of the tally slabs: the binned flux tally's and the reaction rates'.
static inline size_t slab_bytes(const GeomDev &g, const TallyDev &t)
{
    if (!t.enabled) return 0;
    size_t bins = g.tally_kind == TALLY_MESH ? 0 : (size_t)t.n_bins;
    if (t.chan && (size_t)t.chan_bins > bins) bins = (size_t)t.chan_bins;
    return (size_t)WAVES * bins * sizeof(double);
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

hipError_t launch_slots_queue(const BankDev &b, const GeomDev &g, const WwDev &W, Counters *ctr, int cur,
                              uint64_t first_pid, uint64_t n_hist, uint64_t seed, uint32_t new_bound,
                              hipStream_t st)
{
    hipLaunchKernelGGL(k_slots_queue, dim3(blocks_for(b.C, TILE)), dim3(WG), 0, st, b, g, W, ctr, cur,
                       first_pid, n_hist, seed);
    // new histories: at most one per slot, and at most new_bound (the
    // histories not yet started)
    const uint32_t nb = new_bound < b.C ? new_bound : b.C;
    if (nb)
        hipLaunchKernelGGL(k_slots_init, dim3(blocks_for(nb, WG)), dim3(WG), 0, st, b, g, W, ctr, cur, first_pid, seed);
    return hipGetLastError();
}

hipError_t launch_sort(const XsDev &xs, const uint32_t *list, const uint32_t *n_ptr, uint32_t n_bound,
                       const double *E, const int32_t *mat, const SortBufs &sb, uint32_t n_keys,
                       uint32_t *out_list, uint32_t *out_keys, hipStream_t st)
{
    if (n_bound == 0) return hipSuccess;
    uint32_t bits = 1;
    while (bits < 32 && (1ull << bits) < (uint64_t)n_keys) ++bits;
    const int passes = (int)((bits + 7) / 8);
    // the most tiles a queue of up to n_bound keys takes: one per 256 keys
    // up to 2^18 keys, then at most 1024 (a tile holds up to 16 keys per
    // thread) up to 2^22, then one per 4096 keys
    const uint32_t per16 = 16u * 1024u * WG;
    const unsigned tiles = n_bound <= 1024u * WG ? (n_bound + WG - 1) / WG
                           : (n_bound <= per16 ? 1024u : (n_bound + 16u * WG - 1) / (16u * WG));
    SortPassArgs a{};
    a.xs = xs;
    a.E = E;
    a.mat = mat;
    a.n_ptr = n_ptr;
    a.n_fixed = n_bound;
    a.tile_hist = sb.tile_hist;
    a.chunk_total = sb.chunk_total;
    a.chunk_off = sb.chunk_off;
    for (int p = 0; p < passes; ++p) {
        a.shift = 8 * p;
        if (p == 0) {
            a.keys_in = nullptr;
            a.keys_first = sb.kA;
            a.vals_in = list;
        } else {
            a.keys_in = (p & 1) ? sb.kB : sb.kA;
            a.keys_first = nullptr;
            a.vals_in = (p & 1) ? sb.vB : sb.vA;
        }
        if (p == passes - 1) {
            a.keys_out = out_keys;
            a.vals_out = out_list;
        } else {
            a.keys_out = (p & 1) ? sb.kA : sb.kB;
            a.vals_out = (p & 1) ? sb.vA : sb.vB;
        }
        hipLaunchKernelGGL(k_radix_count, dim3(tiles), dim3(WG), 0, st, a);
        hipLaunchKernelGGL(k_radix_scan, dim3(1), dim3(WG), 0, st, sb.chunk_total, sb.chunk_off, n_ptr, n_bound);
        hipLaunchKernelGGL(k_radix_scatter, dim3(tiles), dim3(WG), 0, st, a);
    }
    return hipGetLastError();
}

hipError_t launch_lookup_mp(const MpDev &mp, uint32_t n, const double *E, const int32_t *mat, double *Sa,
                            double *Ss, unsigned long long *pole_count, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_lookup_mp, dim3(blocks_for(n, WG)), dim3(WG), 0, st, mp, n, E, mat, Sa, Ss, pole_count);
    return hipGetLastError();
}

// bounds over every shape of a sort of at most n keys (one key per thread)
size_t sort_tile_count(size_t n) { return (n + WG - 1) / WG; }
size_t sort_chunk_count(size_t n) { return sort_tile_count(n) / 16 + 1; }

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
    a.cp = l.cp;
    a.sx = l.sx;
    const dim3 grid(blocks_for(l.n_bound, WG));
    if (l.xs.um && !(a.sx && l.xs.n_chan > 0) && !(a.idx_out || a.sc_out || a.ss_out)) {
        switch (l.ilp) {  // unionized grid
        case 1: hipLaunchKernelGGL(k_lookup_union<1>, grid, dim3(WG), 0, st, a); break;
        case 2: hipLaunchKernelGGL(k_lookup_union<2>, grid, dim3(WG), 0, st, a); break;
        default: hipLaunchKernelGGL(k_lookup_union<4>, grid, dim3(WG), 0, st, a); break;
        }
    } else if (a.sx && l.xs.n_chan > 0) {  // channels: at most two nuclides in lockstep (registers)
        if (a.keys) hipLaunchKernelGGL((k_lookup<2, false, true, true>), grid, dim3(WG), 0, st, a);
        else if (l.ilp == 1) hipLaunchKernelGGL((k_lookup<1, false, true>), grid, dim3(WG), 0, st, a);
        else hipLaunchKernelGGL((k_lookup<2, false, true>), grid, dim3(WG), 0, st, a);
    } else if (a.idx_out || a.sc_out || a.ss_out) {
        switch (l.ilp) {
        case 1: hipLaunchKernelGGL((k_lookup<1, true, false>), grid, dim3(WG), 0, st, a); break;
        case 2: hipLaunchKernelGGL((k_lookup<2, true, false>), grid, dim3(WG), 0, st, a); break;
        default: hipLaunchKernelGGL((k_lookup<4, true, false>), grid, dim3(WG), 0, st, a); break;
        }
    } else {
        if (a.keys) {  // sorted: staged workgroups read shared grid windows
            hipLaunchKernelGGL((k_lookup<2, false, false, true>), grid, dim3(WG), 0, st, a);
        } else {
            switch (l.ilp) {
            case 1: hipLaunchKernelGGL((k_lookup<1, false, false>), grid, dim3(WG), 0, st, a); break;
            case 2: hipLaunchKernelGGL((k_lookup<2, false, false>), grid, dim3(WG), 0, st, a); break;
            default: hipLaunchKernelGGL((k_lookup<4, false, false>), grid, dim3(WG), 0, st, a); break;
            }
        }
    }
    return hipGetLastError();
}

hipError_t launch_advance(const BankDev &b, const GeomDev &g, const TallyDev &t, const WwDev &W, const Counters *ctr,
                          uint32_t n_bound, uint64_t seed, int64_t max_events, int32_t log_on, bool cross,
                          HistLog *log, uint64_t first_pid, unsigned long long *lost, hipStream_t st)
{
    if (n_bound == 0) return hipSuccess;
    const size_t lds = slab_bytes(g, t);
    const dim3 grid(blocks_for(n_bound, WG));
    const bool lg = log != nullptr || log_on != 0;
    if (cross && lg)
        hipLaunchKernelGGL((k_advance<true, true>), grid, dim3(WG), lds, st, b, g, t, W, ctr, seed, max_events, log_on,
                           log, first_pid, lost);
    else if (cross)
        hipLaunchKernelGGL((k_advance<true, false>), grid, dim3(WG), lds, st, b, g, t, W, ctr, seed, max_events,
                           log_on, log, first_pid, lost);
    else if (lg)
        hipLaunchKernelGGL((k_advance<false, true>), grid, dim3(WG), lds, st, b, g, t, W, ctr, seed, max_events,
                           log_on, log, first_pid, lost);
    else
        hipLaunchKernelGGL((k_advance<false, false>), grid, dim3(WG), lds, st, b, g, t, W, ctr, seed, max_events,
                           log_on, log, first_pid, lost);
    return hipGetLastError();
}

hipError_t launch_split(const BankDev &b, Counters *ctr, uint32_t n_bound, hipStream_t st)
{
    const unsigned nt = blocks_for(n_bound > 0 ? n_bound : 1, TILE);
    hipLaunchKernelGGL(k_split_count, dim3(nt), dim3(WG), 0, st, b, ctr);
    hipLaunchKernelGGL(k_split_scatter, dim3(nt), dim3(WG), 0, st, b, ctr);
    return hipGetLastError();
}

hipError_t launch_cross(const BankDev &b, const GeomDev &g, const TallyDev &t, const WwDev &W, const Counters *ctr,
                        uint32_t n_bound, uint64_t seed, HistLog *log, uint64_t first_pid, unsigned long long *lost,
                        hipStream_t st)
{
    if (n_bound == 0) return hipSuccess;
    const dim3 grid(blocks_for(n_bound, WG));
    switch (W.kind) {
    case WW_LINEAR:
        hipLaunchKernelGGL(k_cross<WW_LINEAR>, grid, dim3(WG), 0, st, b, g, t, W, ctr, seed, log, first_pid, lost);
        break;
    case WW_MLP:
        hipLaunchKernelGGL(k_cross<WW_MLP>, grid, dim3(WG), 0, st, b, g, t, W, ctr, seed, log, first_pid, lost);
        break;
    default:
        hipLaunchKernelGGL(k_cross<WW_OFF>, grid, dim3(WG), 0, st, b, g, t, W, ctr, seed, log, first_pid, lost);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_collide(const BankDev &b, const uint32_t *list, const XsDev &xs, const GeomDev &g,
                          const TallyDev &t, const WwDev &W, const Counters *ctr, uint32_t n_bound, uint64_t seed,
                          HistLog *log, uint64_t first_pid, hipStream_t st)
{
    if (n_bound == 0) return hipSuccess;
    const size_t lds = slab_bytes(g, t);
    const dim3 grid(blocks_for(n_bound, WG));
    const bool lg = log != nullptr;
    switch (W.kind) {
    case WW_LINEAR:
        if (lg)
            hipLaunchKernelGGL((k_collide<WW_LINEAR, true>), grid, dim3(WG), lds, st, b, list, xs, g, t, W, ctr, seed,
                               log, first_pid);
        else
            hipLaunchKernelGGL((k_collide<WW_LINEAR, false>), grid, dim3(WG), lds, st, b, list, xs, g, t, W, ctr,
                               seed, log, first_pid);
        break;
    case WW_MLP:
        if (lg)
            hipLaunchKernelGGL((k_collide<WW_MLP, true>), grid, dim3(WG), lds, st, b, list, xs, g, t, W, ctr, seed, log,
                               first_pid);
        else
            hipLaunchKernelGGL((k_collide<WW_MLP, false>), grid, dim3(WG), lds, st, b, list, xs, g, t, W, ctr, seed,
                               log, first_pid);
        break;
    default:
        if (lg)
            hipLaunchKernelGGL((k_collide<WW_OFF, true>), grid, dim3(WG), lds, st, b, list, xs, g, t, W, ctr, seed, log,
                               first_pid);
        else
            hipLaunchKernelGGL((k_collide<WW_OFF, false>), grid, dim3(WG), lds, st, b, list, xs, g, t, W, ctr, seed,
                               log, first_pid);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_tail(const BankDev &b, const XsDev &xs, const GeomDev &g, const TallyDev &t, const Counters *ctr,
                       uint32_t n_bound, uint64_t seed, int64_t max_events, HistLog *log, uint64_t first_pid,
                       unsigned long long *lost, hipStream_t st)
{
    if (n_bound == 0) return hipSuccess;
    const size_t lds = slab_bytes(g, t);
    if (t.chan)
        hipLaunchKernelGGL(k_tail<true>, dim3(blocks_for(n_bound, WG)), dim3(WG), lds, st, b, xs, g, t, ctr, seed,
                           max_events, log, first_pid, lost);
    else
        hipLaunchKernelGGL(k_tail<false>, dim3(blocks_for(n_bound, WG)), dim3(WG), lds, st, b, xs, g, t, ctr, seed,
                           max_events, log, first_pid, lost);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// weight-window copies: stacks -> copy bank, in slot order
// ---------------------------------------------------------------------------
// Exclusive prefix of v over the workgroup's threads and the total.
__device__ __forceinline__ uint32_t block_exscan_u32(uint32_t v, uint32_t *lds, uint32_t &total)
{
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) lds[wave] = x;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) {
        const uint32_t c = lds[w];
        pre += (w < wave) ? c : 0u;
        tot += c;
    }
    __syncthreads();
    total = tot;
    return pre + x - v;
}

__global__ void __launch_bounds__(WG) k_ww_flush_count(BankDev b, WwDev W)
{
    __shared__ uint32_t lds[32];
    const uint32_t base = blockIdx.x * (uint32_t)TILE;
    uint32_t c = 0;
    for (int r = 0; r < TILE_ITEMS; ++r) {
        const uint32_t s = base + r * WG + threadIdx.x;
        if (s < b.C) c += ww_pending_copies(W, s);
    }
    block_count3(c, 0u, 0u, lds, b.tile_cnt + blockIdx.x * 3);
}

// Every slot's pending copies go to the bank at top + (copies of the slots
// before it), unless they would not all fit: then every stack keeps its own.
__global__ void __launch_bounds__(WG) k_ww_flush_scatter(BankDev b, WwDev W, Counters *ctr)
{
    __shared__ uint32_t lds[32];
    const uint32_t n_tiles = (b.C + TILE - 1) / TILE;
    uint32_t pre[3], tot[3];
    tile_prefix3(b.tile_cnt, n_tiles, blockIdx.x, lds, pre, tot);
    const uint32_t top = ctr->top;
    const bool fits = (uint64_t)top + tot[0] <= (uint64_t)W.Q;
    if (blockIdx.x == 0 && threadIdx.x == 0) ctr->top_after = fits ? top + tot[0] : top;
    // nothing to move, or nothing in this tile (its count is uniform over the block)
    if (!fits || tot[0] == 0 || b.tile_cnt[blockIdx.x * 3] == 0) return;
    const uint32_t base = blockIdx.x * (uint32_t)TILE;
    uint32_t run = 0;
    for (int r = 0; r < TILE_ITEMS; ++r) {
        const uint32_t s = base + r * WG + threadIdx.x;
        const uint32_t c = s < b.C ? ww_pending_copies(W, s) : 0u;
        uint32_t round_total;
        const uint32_t off = block_exscan_u32(c, lds, round_total);
        if (c) ww_flush_slot(W, s, b.pid[s], top + pre[0] + run + off);
        run += round_total;
    }
}

hipError_t launch_ww_flush(const BankDev &b, const WwDev &W, Counters *ctr, hipStream_t st)
{
    const unsigned nt = blocks_for(b.C, TILE);
    hipLaunchKernelGGL(k_ww_flush_count, dim3(nt), dim3(WG), 0, st, b, W);
    hipLaunchKernelGGL(k_ww_flush_scatter, dim3(nt), dim3(WG), 0, st, b, W, ctr);
    return hipGetLastError();
}

// ln I at the source point (one lane), for the windows of the next batch
__global__ void __launch_bounds__(WG) k_ww_source(WwDev W, GeomDev g, double *out)
{
    double x = g.src_pos[0], y = g.src_pos[1], z = g.src_pos[2];
    if (g.src_kind == SRC_BOX) {
        x = 0.5 * (g.src_box[0] + g.src_box[1]);
        y = 0.5 * (g.src_box[2] + g.src_box[3]);
        z = 0.5 * (g.src_box[4] + g.src_box[5]);
    }
    Particle p{};
    p.x = x; p.y = y; p.z = z;
    p.E = g.src_E;
    double v = 0.0;
    if (W.kind == WW_LINEAR) v = ww_ln_importance<WW_LINEAR>(W, p, true);
    else v = ww_ln_importance<WW_MLP>(W, p, threadIdx.x == 0);
    if (threadIdx.x == 0) *out = v;
}

hipError_t launch_ww_source(const WwDev &W, const GeomDev &g, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_ww_source, dim3(1), dim3(WG), 0, st, W, g, out);
    return hipGetLastError();
}

hipError_t launch_problem_set(const SetDev &set, const XsDev &xs, int64_t max_events, uint32_t grid,
                              int32_t max_bins, hipStream_t st)
{
    // the queue counter and the tile rows start at zero (fill kernels: the
    // sequence may be captured into a graph)
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(WG), 0, st, set.next_tile, (size_t)1, 0u);
    unsigned g1 = blocks_for(set.n_rows_doubles, WG);
    if (g1 > 4096) g1 = 4096;
    hipLaunchKernelGGL(k_fill_f64, dim3(g1), dim3(WG), 0, st, set.tl, set.n_rows_doubles, 0.0);
    hipLaunchKernelGGL(k_fill_f64, dim3(g1), dim3(WG), 0, st, set.coll, set.n_rows_doubles, 0.0);
    unsigned g2 = blocks_for((size_t)set.n_tiles * N_GLOBAL, WG);
    if (g2 > 4096) g2 = 4096;
    hipLaunchKernelGGL(k_fill_f64, dim3(g2), dim3(WG), 0, st, set.glob, (size_t)set.n_tiles * N_GLOBAL, 0.0);
    const size_t lds = (size_t)WAVES * (size_t)max_bins * sizeof(double);
    hipLaunchKernelGGL(k_problem_set, dim3(grid), dim3(WG), lds, st, set, xs, max_events);
    hipLaunchKernelGGL(k_problem_set_stats, dim3(set.n_problems), dim3(WG), 0, st, set);
    hipLaunchKernelGGL(k_problem_set_next, dim3(1), dim3(1), 0, st, set);
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

hipError_t launch_batch_accum_strided(const double *T, int32_t n_b, int32_t stride, int32_t off, int32_t n_cols,
                                      double *S1, double *S2, hipStream_t st)
{
    if (n_cols == 0 || n_b == 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_accum, dim3(blocks_for(n_cols, WG)), dim3(WG), 0, st, T, n_b, stride, off, n_cols,
                       S1, S2);
    return hipGetLastError();
}

}  // namespace mc
