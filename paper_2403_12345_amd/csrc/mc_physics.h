// mc_physics.h -- one implementation of the per-particle steps of the
// transport loop (lookup, flight, surface crossing, collision) and of the
// deterministic workgroup tally accumulation.  The event kernels load a
// particle from the bank, call one step and store what changed; the tile
// kernel keeps the particle in registers and calls the steps in a loop.  Both
// therefore produce the same history for the same particle.
#pragma once

#include "mc_device.h"

#pragma clang fp contract(off)

namespace mc {

// ---------------------------------------------------------------------------
// particle state in registers
// ---------------------------------------------------------------------------
struct Particle {
    double x, y, z, u, v, w, E, wt, Sa, Ss, track;
    uint64_t pid;
    uint32_t ndraw, lineage;
    int32_t mat, cell, ncoll, ncross;
    bool inside;
    uint8_t ev;
};

__device__ __forceinline__ Particle load_particle(const BankDev &b, uint32_t s)
{
    Particle p;
    p.x = b.x[s]; p.y = b.y[s]; p.z = b.z[s];
    p.u = b.u[s]; p.v = b.v[s]; p.w = b.w[s];
    p.E = b.E[s]; p.wt = b.wt[s]; p.Sa = b.Sa[s]; p.Ss = b.Ss[s]; p.track = b.track[s];
    p.pid = b.pid[s]; p.ndraw = b.ndraw[s]; p.lineage = b.lineage[s];
    p.mat = b.mat[s]; p.cell = b.cell[s]; p.ncoll = b.ncoll[s]; p.ncross = b.ncross[s];
    p.inside = b.inside[s] != 0;
    p.ev = b.event[s];
    return p;
}

// What one step adds to the tallies of its workgroup.
struct StepScore {
    int32_t tl_bin;   // track-length flux bin (-1: none)
    double tl_val;
    int32_t c_bin;    // collision-estimator bin (-1: none)
    double c_val;
    double g[N_GLOBAL];
};

__device__ __forceinline__ void clear_score(StepScore &sc)
{
    sc.tl_bin = -1; sc.tl_val = 0.0;
    sc.c_bin = -1; sc.c_val = 0.0;
#pragma unroll
    for (int k = 0; k < N_GLOBAL; ++k) sc.g[k] = 0.0;
}

__device__ __forceinline__ void write_log(HistLog *log, uint64_t first_pid, const Particle &p, int32_t fate)
{
    HistLog h;
    h.fate = fate;
    h.n_coll = p.ncoll;
    h.n_cross = p.ncross;
    h.pad = 0;
    h.n_draws = p.ndraw;
    h.E_final = p.E;
    h.track = p.track;
    h.weight = p.wt;
    log[p.pid - first_pid] = h;
}

// ---------------------------------------------------------------------------
// tally binning
// ---------------------------------------------------------------------------
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

// Track-length score of a straight flight through the mesh: the part of the
// flight inside the mesh box (slab intersection: the entry and exit of the
// flight through each pair of box planes), walked cell by cell by a 3-D
// digital differential analyser, adding w * length per cell.  Track outside
// the box scores nothing.  Distances to planes are divided by the direction
// component as written (a product with its reciprocal would cut the flight
// into extra slivers of a few ulps where a plane's distance and the box's
// clip round apart); cell sizes come precomputed with the geometry.
__device__ inline void mesh_flight(const GeomDev &g, double *acc, double x, double y, double z, double u,
                                   double v, double w, double d, double wt)
{
    const double r0[3] = {x, y, z}, dir[3] = {u, v, w};
    // [t_in, t_out): the flight's parameter range inside the box
    double t_in = 0.0, t_out = d;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (dir[k] == 0.0) {
            if (r0[k] < g.mesh_lo[k] || r0[k] > g.mesh_hi[k]) return;
        } else {
            const double ta = (g.mesh_lo[k] - r0[k]) / dir[k], tb = (g.mesh_hi[k] - r0[k]) / dir[k];
            t_in = fmax(t_in, fmin(ta, tb));
            t_out = fmin(t_out, fmax(ta, tb));
        }
    }
    if (!(t_out > t_in)) return;
    double tnext[3], tdelta[3];
    int32_t c[3], step[3];
    // first cell: the one holding the clipped flight's first point (nudged
    // along the flight by a hair so a start on a mesh plane picks the cell ahead)
    const double tq = t_in + fmin(t_out - t_in, 1e-9) * 0.5;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double h = g.mesh_h[k];
        const double q = r0[k] + dir[k] * tq;
        int32_t v0 = (int32_t)floor((q - g.mesh_lo[k]) / h);
        c[k] = v0 < 0 ? 0 : (v0 > g.mesh_dims[k] - 1 ? g.mesh_dims[k] - 1 : v0);
        if (dir[k] > 0.0) {
            step[k] = 1;
            tnext[k] = (g.mesh_lo[k] + (c[k] + 1) * h - r0[k]) / dir[k];
            tdelta[k] = h / dir[k];
        } else if (dir[k] < 0.0) {
            step[k] = -1;
            tnext[k] = (g.mesh_lo[k] + c[k] * h - r0[k]) / dir[k];
            tdelta[k] = -h / dir[k];
        } else {
            step[k] = 0;
            tnext[k] = INFINITY;
            tdelta[k] = INFINITY;
        }
    }
    // the mesh sizes in registers: indexed by the axis of the step, the
    // argument array would be read from memory each step, and that read
    // would wait for the step's atomic add to complete
    const int32_t nx = g.mesh_dims[0], ny = g.mesh_dims[1], nz = g.mesh_dims[2];
    double t = t_in;
    for (int guard = 0; guard < 100000 && t < t_out; ++guard) {
        int k = 0;
        if (tnext[1] < tnext[k]) k = 1;
        if (tnext[2] < tnext[k]) k = 2;
        const double t1 = fmin(fmax(tnext[k], t), t_out);
        if (t1 > t) {
            const int32_t idx = (c[2] * ny + c[1]) * nx + c[0];
            mesh_add(acc, idx, wt * (t1 - t), g.n_bins);
        }
        t = t1;
        if (t >= t_out) break;
        c[k] += step[k];
        const int32_t nk = k == 0 ? nx : (k == 1 ? ny : nz);
        if (c[k] < 0 || c[k] >= nk) break;
        tnext[k] += tdelta[k];
    }
}

// ---------------------------------------------------------------------------
// deterministic workgroup accumulation (no atomics)
// ---------------------------------------------------------------------------
// Adds val into bin `bin` (< 0: nothing) of the workgroup's row.  Each wave
// peels off one distinct bin at a time: the values of the lanes holding it
// are added in lane order when they are few (cheaper than a reduction over
// all 64), by the wave's DPP reduction tree when they are many, and the first of them adds
// the sum into the wave's LDS slab;
// the slabs are then added in wave order into the row.  Every thread of the
// workgroup must call it.
__device__ __forceinline__ double lanes_sum(double v, uint64_t lanes)
{
    // many lanes (a material's rates, one bin per wave): the DPP tree over
    // the whole wave (every lane of the wave is active here)
    if (__popcll(lanes) > 8) return wave_sum(((lanes >> lane_id()) & 1ull) ? v : 0.0);
    double s = 0.0;
    while (lanes) {
        const int j = __ffsll((long long)lanes) - 1;
        s = s + lane_f64(v, j);
        lanes &= lanes - 1ull;
    }
    return s;
}

__device__ inline void wg_bin_add(int32_t bin, double val, double *slab, int32_t nbins, double *row)
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
        const double s = lanes_sum(val, __ballot(mine));
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

// Adds the per-thread global-tally values into the workgroup's row (every
// thread must call it; lds holds N_GLOBAL * WAVES doubles).
__device__ inline void wg_glob_add(const double (&val)[N_GLOBAL], double *lds, double *row)
{
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < N_GLOBAL; ++k) {
        // a wave whose lanes all hold zero for this sum skips the reduction
        // (its slot is zero either way): each event kernel scores only a few
        // of the sums, and those it never touches are dropped when compiled
        const double s = __ballot(val[k] != 0.0) ? wave_sum(val[k]) : 0.0;
        if (lane_id() == 0) lds[k * WAVES + wave] = s;
    }
    __syncthreads();
    if (threadIdx.x < N_GLOBAL) {
        double s = 0.0;
        for (int w = 0; w < WAVES; ++w) s = s + lds[threadIdx.x * WAVES + w];
        if (s != 0.0) row[threadIdx.x] = row[threadIdx.x] + s;
    }
    __syncthreads();
}

// Adds each lane's track-length reaction rates wd * sx[x] (x < K) into the
// workgroup's row [n_mat][K] at its flight's material (mat < 0: no flight).
// Every thread must call it; slab holds WAVES * nb doubles, nb = n_mat * K.
__device__ inline void wg_chan_add(int32_t mat, double wd, const double *sx, int32_t K, double *slab, int32_t nb,
                                   double *row)
{
    for (int32_t t = threadIdx.x; t < WAVES * nb; t += WG) slab[t] = 0.0;
    __syncthreads();
    const int wave = threadIdx.x >> 6;
    bool active = mat >= 0;
    uint64_t mask = __ballot(active);
    while (mask) {
        const int leader = __ffsll((long long)mask) - 1;
        const int32_t M = __shfl(mat, leader, 64);
        const bool mine = active && mat == M;
        const uint64_t lanes = __ballot(mine);
        for (int32_t x = 0; x < K; ++x) {
            const double s = lanes_sum(wd * sx[x], lanes);
            if (lane_id() == leader) slab[wave * nb + M * K + x] += s;
        }
        active = active && !mine;
        mask = __ballot(active);
    }
    __syncthreads();
    for (int32_t t = threadIdx.x; t < nb; t += WG) {
        double s = 0.0;
        for (int w = 0; w < WAVES; ++w) s = s + slab[w * nb + t];
        if (s != 0.0) row[t] = row[t] + s;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// the steps
// ---------------------------------------------------------------------------
constexpr int DEFAULT_LOOKUP_ILP = 2;

// Macroscopic cross sections of the particle's material at its energy
// (hash brackets read from global memory); CHAN: also the reaction channels
// into sx_row; cp_row (nullable): the scattering-sum checkpoints, as the
// event-loop lookup writes them.
template <int ILP, bool CHAN = false>
__device__ inline void do_lookup(Particle &p, const XsDev &xs, double *sx_row = nullptr, double *cp_row = nullptr)
{
    const int32_t q0 = xs.mat_off[p.mat], nk = xs.mat_off[p.mat + 1] - q0;
    const int32_t bin = hash_bin(xs, p.E);
    const float tb = bin_position(xs, p.E, bin);
    const uint2 *h = hash_row(xs, p.mat, bin, nk);
    double sa = 0.0, ss = 0.0;
    const int32_t cp_sh = cp_row && nk > CP_MIN_NUC ? cp_shift(nk) : 30;  // 30: never a checkpoint
    const int32_t cp_mask = (1 << cp_sh) - 1;
    CpPairs cpw{cp_row, 0.0};
    double acc[MAX_CHAN];
    if (CHAN) {
#pragma unroll
        for (int x = 0; x < MAX_CHAN; ++x) acc[x] = 0.0;
    }
    for (int32_t q = 0; q < nk; q += ILP) {
        const int32_t cnt = nk - q < ILP ? nk - q : ILP;
        double dens[ILP], c[ILP], s[ILP], fr[ILP];
        uint32_t ix[ILP], pt[ILP];
        micro_group<ILP>(xs, xs.mnuc + q0, h, nk, q, cnt, p.E, tb, dens, ix, c, s, fr, pt);
        if (CHAN) channel_group<ILP>(xs, cnt, dens, fr, pt, acc);
#pragma unroll
        for (int k = 0; k < ILP; ++k) {
            if (k < cnt) {
                sa = sa + dens[k] * c[k];
                ss = ss + dens[k] * s[k];
                const int32_t done = q + k + 1;
                if ((done & cp_mask) == 0) cpw.put((done >> cp_sh) - 1, ss);
            }
        }
    }
    if (cp_sh != 30) cpw.finish(nk >> cp_sh);
    p.Sa = sa;
    p.Ss = ss;
    if (CHAN) {
#pragma unroll
        for (int x = 0; x < MAX_CHAN; ++x)
            if (x < xs.n_chan) sx_row[x] = acc[x];
    }
}

// Flight: distance to collision -ln(xi)/Sigma_t (one draw), distance to the
// nearest surface, move by the smaller, score the track length.  Sets p.ev
// and returns the flight's length.  A mesh tally with mesh_tl null is left to
// the caller (mesh_flight from the flight's start).
__device__ inline double do_advance(Particle &p, const GeomDev &g, uint64_t seed, bool tally_on, double *mesh_tl,
                                    bool log_on, StepScore &sc)
{
    Rng rng(seed, p.pid, p.lineage, p.ndraw);
    const double st = p.Sa + p.Ss;
    const double dc = -log(rng.next()) / st;
    uint8_t ev;
    const double db = surface_distance(g, p.x, p.y, p.z, p.u, p.v, p.w, p.cell, p.inside, ev);
    const double d = (db < dc) ? db : dc;
    if (!(db < dc)) ev = EV_COLLIDE;
    const double x0 = p.x, y0 = p.y, z0 = p.z;
    p.x = p.x + d * p.u;
    p.y = p.y + d * p.v;
    p.z = p.z + d * p.w;
    p.ndraw = rng.n;
    p.ev = ev;
    if (log_on) p.track = p.track + d;
    sc.g[G_TRACK] += p.wt * d;
    sc.g[G_TRACK_ABS] += p.wt * d * p.Sa;
    if (tally_on) {
        switch (g.tally_kind) {
        case TALLY_ENERGY: sc.tl_bin = energy_bin(g, p.E); break;
        case TALLY_PIN: sc.tl_bin = p.inside ? p.cell : -1; break;
        case TALLY_SLAB: sc.tl_bin = p.cell; break;
        case TALLY_MESH:
            if (mesh_tl) mesh_flight(g, mesh_tl, x0, y0, z0, p.u, p.v, p.w, d, p.wt);
            break;
        }
        sc.tl_val = p.wt * d;
    }
    return d;
}

// Surface crossing p.ev: lattice step (the coordinate snaps onto the plane),
// cylinder sense, reflection or leakage at an outer face.  Returns
// FATE_LEAKED or 0; need_lookup tells whether the material changed, leak_xhi
// whether the particle leaked through the x+ face.
__device__ inline int32_t do_cross(Particle &p, const GeomDev &g, StepScore &sc, bool &need_lookup, bool &leak_xhi)
{
    need_lookup = false;
    leak_xhi = false;
    sc.g[G_NCROSS] += 1.0;
    p.ncross += 1;
    int32_t cell = p.cell;
    bool inside = p.inside;
    int face = -1;  // outer face reached (0..5 = x-, x+, y-, y+, z-, z+)
    double face_pos = 0.0;
    if (g.kind == GEOM_SLAB) {
        if (p.ev == EV_XHI) {
            if (cell == g.n_layers - 1) { face = 1; face_pos = g.x_edges[g.n_layers]; }
            else { cell += 1; p.x = g.x_edges[cell]; }
        } else {
            if (cell == 0) { face = 0; face_pos = g.x_edges[0]; }
            else { p.x = g.x_edges[cell]; cell -= 1; }
        }
    } else {
        const int32_t ci = cell % g.nx, cj = cell / g.nx;
        const double P = g.pitch;
        switch (p.ev) {
        case EV_CYL: inside = !inside; break;
        case EV_XHI:
            if (ci == g.nx - 1) { face = 1; face_pos = (double)g.nx * P; }
            else { cell += 1; p.x = (double)(ci + 1) * P; }
            break;
        case EV_XLO:
            if (ci == 0) { face = 0; face_pos = 0.0; }
            else { p.x = (double)ci * P; cell -= 1; }
            break;
        case EV_YHI:
            if (cj == g.ny - 1) { face = 3; face_pos = (double)g.ny * P; }
            else { cell += g.nx; p.y = (double)(cj + 1) * P; }
            break;
        case EV_YLO:
            if (cj == 0) { face = 2; face_pos = 0.0; }
            else { p.y = (double)cj * P; cell -= g.nx; }
            break;
        case EV_ZHI: face = 5; face_pos = g.z1; break;
        case EV_ZLO: face = 4; face_pos = g.z0; break;
        default: break;
        }
    }
    if (face >= 0) {
        // (the face's condition picked from the six, not indexed: an indexed
        // read of the argument array would go to memory)
        int32_t bcf = g.bc[0];
#pragma unroll
        for (int f = 1; f < 6; ++f) bcf = face == f ? g.bc[f] : bcf;
        if (bcf == BC_VACUUM) {
            sc.g[G_LEAK] += p.wt;
            if (face == 1) {
                leak_xhi = true;
                sc.g[G_LEAK_XHI] += p.wt;
                if (p.ncoll == 0) sc.g[G_LEAK_XHI_UNC] += p.wt;
            }
            return FATE_LEAKED;
        }
        const int axis = face >> 1;
        if (axis == 0) { p.u = -p.u; p.x = face_pos; }
        else if (axis == 1) { p.v = -p.v; p.y = face_pos; }
        else { p.w = -p.w; p.z = face_pos; }
    }
    const int32_t m_new = region_material(g, cell, inside);
    p.cell = cell;
    p.inside = inside;
    if (m_new != p.mat) {
        p.mat = m_new;
        need_lookup = true;
    }
    return 0;
}

// Collision: collision estimator; analog capture when xi * Sigma_t < Sigma_a;
// otherwise the target is the first nuclide whose running sum of
// density * sigma_s reaches xi * Sigma_s (sigma_s gathered again, material
// order; with checkpoints of that running sum from the particle's lookup --
// cp != nullptr, the particle's row -- the walk starts at the last checkpoint
// below the target, with the same partial sum), elastic scattering off it at
// rest with an isotropic centre-of-mass cosine, and the energy cutoff.
// Returns FATE_ABSORBED, FATE_CUTOFF or 0.
template <int CILP = DEFAULT_LOOKUP_ILP>
__device__ inline int32_t do_collide(Particle &p, const XsDev &xs, const GeomDev &g, uint64_t seed,
                                     bool tally_on, double *mesh_coll, StepScore &sc, const double *cp)
{
    const double st = p.Sa + p.Ss;
    p.ncoll += 1;
    sc.g[G_NCOLL] += 1.0;
    sc.g[G_COLL_EST] += p.wt / st;
    if (tally_on) {
        switch (g.tally_kind) {
        case TALLY_ENERGY: sc.c_bin = energy_bin(g, p.E); break;
        case TALLY_PIN: sc.c_bin = p.inside ? p.cell : -1; break;
        case TALLY_SLAB: sc.c_bin = p.cell; break;
        case TALLY_MESH: {  // (mesh_coll null: the caller scores it)
            const int32_t c = mesh_coll ? mesh_index(g, p.x, p.y, p.z) : -1;
            if (c >= 0) mesh_add(mesh_coll, c, p.wt / st, g.n_bins);
        } break;
        }
        sc.c_val = p.wt / st;
    }
    Rng rng(seed, p.pid, p.lineage, p.ndraw);
    if (rng.next() * st < p.Sa) {
        sc.g[G_ABSORB] += p.wt;
        p.ndraw = rng.n;
        return FATE_ABSORBED;
    }
    const double target = rng.next() * p.Ss;
    const int32_t q0 = xs.mat_off[p.mat], nk = xs.mat_off[p.mat + 1] - q0;
    const int32_t bin = hash_bin(xs, p.E);
    const float tb = bin_position(xs, p.E, bin);
    const uint2 *h = hash_row(xs, p.mat, bin, nk);
    double cum = 0.0;
    int32_t pick = -1, qstart = 0;
    const int32_t ncp = cp ? cp_count(nk) : 0;
    if (ncp > 0) {
        // the first checkpoint at or above the target bounds the segment:
        // checkpoints never decrease, so its index is the count of those below
        // the target; the row (16-byte pairs) is read in one round of loads
        int32_t j = 0;
#pragma unroll
        for (int32_t k = 0; k < CP_MAX; k += 2) {
            if (k < ncp) {
                const double2 v = *reinterpret_cast<const double2 *>(cp + k);
                j += v.x < target ? 1 : 0;
                j += (k + 1 < ncp && v.y < target) ? 1 : 0;
            }
        }
        if (j > 0) {
            cum = cp[j - 1];
            qstart = j << cp_shift(nk);
        }
    }
    bool done = false;
    for (int32_t q = qstart; q < nk && !done; q += CILP) {
        const int32_t cnt = nk - q < CILP ? nk - q : CILP;
        double dens[CILP], c[CILP], sg[CILP];
        uint32_t ix[CILP];
        micro_group<CILP>(xs, xs.mnuc + q0, h, nk, q, cnt, p.E, tb, dens, ix, c, sg);
#pragma unroll
        for (int k = 0; k < CILP; ++k) {
            if (k < cnt && !done) {
                const double term = dens[k] * sg[k];
                cum = cum + term;
                if (term > 0.0) pick = q + k;
                if (cum >= target && term > 0.0) done = true;
            }
        }
    }
    const double A = xs.awr[xs.mat_nuc[q0 + (pick < 0 ? 0 : pick)]];
    const double mu = 2.0 * rng.next() - 1.0;
    const double phi = 2.0 * M_PI * rng.next();
    double e2, mul;
    elastic_at_rest(A, p.E, mu, e2, mul);
    turn(p.u, p.v, p.w, mul, phi);
    p.E = e2;
    p.ndraw = rng.n;
    if (e2 < g.e_cut) {
        sc.g[G_CUTOFF] += p.wt;
        return FATE_CUTOFF;
    }
    return 0;
}

}  // namespace mc
