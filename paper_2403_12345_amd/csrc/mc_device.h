// mc_device.h -- device-side data layout and per-particle primitives of the
// gfx950 transport path.  Every expression here is compiled with fp
// contraction off (see the pragma below and -ffp-contract=off on the hipcc
// line) so that interpolation, macroscopic sums and kinematics round exactly
// as written.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#pragma clang fp contract(off)

namespace mc {

constexpr int WG = 256;          // threads per workgroup of every event kernel
constexpr int WAVES = WG / 64;   // wave64
constexpr int TILE_ITEMS = 4;    // items per thread in the queue-building kernels
constexpr int TILE = WG * TILE_ITEMS;
constexpr int MAX_LDS_BINS = 1024;  // tallies with more bins use the mesh path

// particle flags
constexpr uint8_t F_ALIVE = 1, F_LOOKUP = 2;
// event codes written by the advance kernel
enum : uint8_t { EV_COLLIDE = 0, EV_CYL = 1, EV_XLO = 2, EV_XHI = 3, EV_YLO = 4, EV_YHI = 5,
                 EV_ZLO = 6, EV_ZHI = 7,
                 EV_DONE = 0xFE };  // the crossing was done by the flight kernel
enum { GEOM_INFINITE = 0, GEOM_LATTICE = 1, GEOM_SLAB = 2 };
enum { BC_REFLECT = 0, BC_VACUUM = 1 };
enum { SRC_POINT = 0, SRC_BOX = 1, SRC_BEAM = 2 };
enum { TALLY_ENERGY = 0, TALLY_PIN = 1, TALLY_MESH = 2, TALLY_SLAB = 3 };
enum { G_TRACK = 0, G_COLL_EST = 1, G_ABSORB = 2, G_CUTOFF = 3, G_LEAK = 4, G_TRACK_ABS = 5,
       G_NCOLL = 6, G_NCROSS = 7, G_LEAK_XHI = 8, G_LEAK_XHI_UNC = 9, G_SPLIT = 10, G_ROULETTE = 11,
       N_GLOBAL = 12 };
enum { FATE_ABSORBED = 1, FATE_CUTOFF = 2, FATE_LEAKED = 3, FATE_LOST = 4, FATE_ROULETTE = 5 };

// One nuclide entry of a material, in material order: where its grid lives
// in the concatenated tables, how long it is, and its atom density.
struct MatNuc {
    uint32_t off;   // first point of the nuclide's grid in Eg / xs
    uint32_t len;   // number of grid points
    double dens;    // atoms / (barn cm)
};

// Cross-section tables in HBM.
//   Eg[p]      fp64 grid energies of every nuclide, concatenated
//   xs[p]      {sigma_c, sigma_s} at the same point (16 B, one load per point)
//   hash       per material m: M rows of n_k uint2 brackets, row b holding
//              (i_q(E_b), i_q(E_b+1)) for the material's nuclides q (bin-major
//              so that one particle's brackets for all its nuclides are
//              contiguous; one 8-byte load per nuclide)
struct XsDev {
    const double *Eg;
    const double2 *xs;
    const double *awr;         // per nuclide
    const int32_t *mat_off;    // [n_mat + 1] into mat_nuc / mnuc
    const int32_t *mat_nuc;    // nuclide ids in material order
    const MatNuc *mnuc;        // per (material, position)
    const uint2 *hash;         // [hash_off[m] + b * nk + q] = (lo_q(E_b), lo_q(E_b+1)): bin b's bracket
    const uint64_t *hash_off;  // [n_mat] start of material m's rows (in pairs)
    int32_t n_mat;
    int32_t M;                 // hash bins
    double ln_emin, inv_delta; // bin b = floor((ln E - ln emin) * inv_delta)
    int32_t div_safe;          // every grid energy in [2^-100, 2^100] (the interval fraction's short division)
    // reaction channels: n_chan values per grid point, point p's at xc[p * n_chan]
    int32_t n_chan;
    const double *xc;
    // unionized grids (null: the per-nuclide hash search only)
    const struct UnionMat *um;
    const double *ug;      // union grids of all materials
    const uint32_t *uh;    // their hash bounds, M + 1 per material
    const uint32_t *ui;    // index rows: nuclide intervals at each union point
};

// Unionized grid of one material: the sorted union U of its nuclides' grids
// (ug[g_off .. g_off + n)), hash bounds uh[h_off + b] = the union index of the
// bin's lower edge (b = 0 .. M), and per union point u the row
// ui[i_off + u * nk + q] = i_q(U_u), the interval of nuclide position q at U_u.
// No nuclide has a grid point strictly between U_u and U_(u+1), so for U_u <= E <
// U_(u+1) that row holds each nuclide's own interval of E.
struct UnionMat {
    uint64_t g_off, i_off;
    uint32_t n, h_off;
};

constexpr int MAX_CHAN = 16;  // most reaction channels

// Mesh tallies accumulate in 64-bit fixed point, 2^-32 per unit (weight * cm):
// integer additions commute, so the sums do not depend on the order in which
// the atomics land and reruns are bitwise identical.  A contribution v is
// rounded to the nearest 2^-32 (absolute error at most 2^-33 per
// contribution).  Range: a bin holds at most 2^64 units, and no bin can
// exceed 2^32 times the batch's total weighted track length plus half a unit
// per contribution, so a batch whose global track total stays below 2^31
// cannot wrap any bin; the host checks that bound after every batch
// (MC_ERANGE).  The array has n_bins bins and one more word: the number of
// positive contributions that rounded to zero (below the resolution).
constexpr double MESH_FIX_SCALE = 4294967296.0;        // 2^32
constexpr double MESH_FIX_INV = 1.0 / 4294967296.0;    // 2^-32
constexpr double MESH_TRACK_LIMIT = 2147483648.0;      // 2^31 weight * cm per batch
__device__ __forceinline__ void mesh_add(double *acc, int32_t idx, double v, int32_t n_bins)
{
    unsigned long long *a = reinterpret_cast<unsigned long long *>(acc);
    const unsigned long long q = __double2ull_rn(v * MESH_FIX_SCALE);
    if (q) atomicAdd(a + idx, q);
    else if (v > 0.0) atomicAdd(a + n_bins, 1ull);
}

struct GeomDev {
    int32_t kind, inf_mat;
    int32_t nx, ny;
    double pitch, radius, z0, z1;
    const int32_t *pin_mat;
    int32_t mod_mat;
    int32_t bc[6];
    int32_t n_layers;
    const double *x_edges;
    const int32_t *layer_mat;
    int32_t src_kind;
    double src_pos[3], src_box[6], src_dir[3], src_E;
    int32_t tally_kind, n_bins, n_ebins;
    const double *e_edges;
    int32_t mesh_dims[3];
    double mesh_lo[3], mesh_hi[3];
    double mesh_h[3];                 // cell size (hi - lo) / dims
    double e_cut;
};

// Structure-of-arrays particle bank (capacity C slots) and its queues.
// Checkpoints of the running sum of N_k sigma_s,k over a material's nuclides
// (material order), written by the lookup for materials of more than
// CP_MIN_NUC nuclides: checkpoint j holds the sum over nuclides
// [0, (j + 1) 2^sh), sh = cp_shift(nk) the smallest shift of at least 3 that
// leaves at most CP_MAX of them.  The collision starts its walk for the
// sampled nuclide at the checkpoint before the target instead of at nuclide
// 0: the same partial sums, far fewer gathers.  (The rows are written by
// scattered stores, two checkpoints at a time, so a few checkpoints per
// lookup, not one per nuclide: each store can cost the lookup a partial-line
// write-back.  For 300 nuclides a stride of 16 (18 checkpoints) beats both 32
// and 8.)
constexpr int CP_MAX = 32, CP_MIN_NUC = 16;
__host__ __device__ __forceinline__ int32_t cp_shift(int32_t nk)
{
    int32_t sh = 3;
    while ((nk >> sh) > CP_MAX) ++sh;
    return sh;
}
__host__ __device__ __forceinline__ int32_t cp_count(int32_t nk)
{
    return nk > CP_MIN_NUC ? nk >> cp_shift(nk) : 0;
}

// The lookup writes a row's checkpoints two at a time (one 16-byte store for
// checkpoints 2i and 2i+1): half as many scattered partial-line writes.
struct CpPairs {
    double *row;  // the particle's row of CP_MAX (16-byte aligned)
    double pend;  // checkpoint 2i, waiting for 2i+1
    __device__ __forceinline__ void put(int32_t j, double v)
    {
        if (j & 1) *reinterpret_cast<double2 *>(row + (j - 1)) = make_double2(pend, v);
        else pend = v;
    }
    // after the last of count checkpoints
    __device__ __forceinline__ void finish(int32_t count)
    {
        if (count & 1) row[count - 1] = pend;
    }
};

struct BankDev {
    double *cp;  // [slot][CP_MAX] checkpoints of the scattering sum (see above): one row per slot
    double *sx;  // [slot][n_chan] macroscopic reaction-channel cross sections (null without channels)
    double *x, *y, *z, *u, *v, *w, *E, *wt, *Sa, *Ss, *track;
    int32_t *mat, *cell, *ncoll, *ncross;
    uint8_t *flags, *inside, *event;
    uint64_t *pid;
    uint32_t *ndraw, *lineage;
    uint32_t *A, *L, *Ls, *Lkey, *Qc, *Qx;   // alive, lookup, sorted lookup, keys, collide, cross
    uint32_t *tile_cnt;                       // per-tile counts of the queue kernels
    uint32_t C;
};

// Queue sizes of one event-loop iteration (a ring of two, by iteration parity).
struct Counters {
    uint64_t issued;   // histories started so far in this batch
    uint32_t nA, nL;   // alive and lookup queue lengths
    uint32_t nC, nX;   // collide and cross queue lengths
    uint32_t n_new;    // source particles started by this iteration's refill
    uint32_t top;      // weight-window copies waiting in the copy bank after the refill
    uint32_t top_after;  // ... and after this iteration's flush
    uint32_t pad;
};

// Per-workgroup tally rows: workgroup g of an event kernel adds its partial
// sums into row g, and only that workgroup writes the row, so no atomics and
// a fixed summation order.
struct TallyDev {
    double *tl;     // [rows][n_bins] track-length flux (lattice / energy / slab)
    double *coll;   // [rows][n_bins] collision estimator
    double *glob;   // [rows][N_GLOBAL]
    double *mesh_tl, *mesh_coll;  // [n_bins] mesh tallies (64-bit fixed point, integer atomics; see mesh_add)
    double *chan;   // [rows][n_mat * n_chan] track-length reaction rates (null without channels)
    int32_t n_chan, chan_bins;
    int32_t n_bins, rows;
    int32_t enabled;  // 0: inactive batch, binned flux tallies off
};

struct HistLog {
    int32_t fate, n_coll, n_cross, pad;
    uint64_t n_draws;
    double E_final, track, weight;
};

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32
// multiplies, a swap-and-xor of the halves with the key, key bumped by the
// golden-ratio / sqrt(3)-1 Weyl increments.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint2 k)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t a0 = 0xD2511F53u * c.x, h0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t a1 = 0xCD9E8D57u * c.z, h1 = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(h1 ^ c.y ^ k.x, a1, h0 ^ c.w ^ k.y, a0);
        k.x += 0x9E3779B9u;
        k.y += 0xBB67AE85u;
    }
    return c;
}

// The stream of one particle: draw n uses counter (n/2, lineage, pid) under
// key seed; even draws take output words (y:x), odd draws (w:z); the top 52
// bits give u = (m + 1/2) 2^-52 in (0, 1).
struct Rng {
    uint64_t seed, pid;
    uint32_t lineage, n;
    uint4 blk;
    bool have;

    __device__ __forceinline__ Rng(uint64_t s, uint64_t p, uint32_t lin, uint32_t n0)
        : seed(s), pid(p), lineage(lin), n(n0), blk(make_uint4(0, 0, 0, 0)), have(false) {}

    __device__ __forceinline__ double next()
    {
        if (!have || (n & 1u) == 0u) {
            blk = philox4x32_10(make_uint4(n >> 1, lineage, (uint32_t)pid, (uint32_t)(pid >> 32)),
                                make_uint2((uint32_t)seed, (uint32_t)(seed >> 32)));
            have = true;
        }
        const uint64_t bits = (n & 1u) ? (((uint64_t)blk.w << 32) | blk.z)
                                       : (((uint64_t)blk.y << 32) | blk.x);
        n += 1;
        return ((double)(bits >> 12) + 0.5) * 0x1p-52;
    }
};

// ---------------------------------------------------------------------------
// cross-section lookup
// ---------------------------------------------------------------------------
__device__ __forceinline__ int32_t hash_bin(const XsDev &xs, double e)
{
    const double t = (log(e) - xs.ln_emin) * xs.inv_delta;
    int32_t b = (t > 0.0) ? (int32_t)t : 0;
    return b < xs.M - 1 ? b : xs.M - 1;
}

// E's position inside hash bin b, in [0, 1]: where a search of the bin's
// bracket starts.  A guide only (the search checks and walks), so single
// precision is enough.
__device__ __forceinline__ float bin_position(const XsDev &xs, double e, int32_t b)
{
    const float t = (__logf((float)e) - (float)xs.ln_emin) * (float)xs.inv_delta - (float)b;
    return fminf(fmaxf(t, 0.f), 1.f);
}

// First probe of a search of the bracket [lo, hi]: the interval nearest to
// the position tb of E inside the bin (grid points of a bin lie roughly
// evenly in ln E).  In the synthetic tables it is the interval sought for
// about 80 % of energies and one off for almost all others.
__device__ __forceinline__ uint32_t bracket_guess(uint32_t lo, uint32_t hi, float tb)
{
    const uint32_t j = lo + (uint32_t)(tb * (float)(hi - lo) + 0.5f);
    return j < hi ? j : hi;
}

// Grid index i(E) = max{j : E_j <= E} clamped to [0, N-2].  [lo, hi] is the
// hash bracket of E's bin; the bisection finds the largest j in it with
// E_j <= E and the two walks then correct for a bin computed one off (the
// device logarithm may round differently from the host's at a bin edge).
__device__ __forceinline__ uint32_t grid_find(const double *__restrict__ g, uint32_t n, uint32_t lo,
                                              uint32_t hi, double e)
{
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1u) >> 1;
        if (g[mid] <= e) lo = mid; else hi = mid - 1u;
    }
    uint32_t i = lo;
    while (i > 0u && e < g[i]) --i;
    while (i + 2u < n && e >= g[i + 1u]) ++i;
    return i;
}

// Micro cross sections of one nuclide at E from interval i (linear in E).
__device__ __forceinline__ void lerp_xs(const XsDev &xs, uint32_t off, uint32_t i, double e,
                                        double &sc, double &ss)
{
    const double e0 = xs.Eg[off + i], e1 = xs.Eg[off + i + 1u];
    const double2 x0 = xs.xs[off + i], x1 = xs.xs[off + i + 1u];
    const double f = (e - e0) / (e1 - e0);
    sc = x0.x + f * (x1.x - x0.x);
    ss = x0.y + f * (x1.y - x0.y);
}

// Micro cross sections of up to ILP nuclides (positions q .. q+cnt-1 of a
// material whose entries start at mnuc, hash bracket pairs h[q]) at E.
// The bisections run in lockstep with their probe loads issued together, so a
// wave keeps ILP independent gathers in flight per step instead of one.  The
// interval found is checked against the energies loaded for the
// interpolation; only when the hash bin was computed one off (device and host
// logarithms rounding differently at a bin edge) does a lane walk to the
// defined index and reload.  Each nuclide's result is exactly that of
// grid_find + lerp_xs.
// Two consecutive grid energies, 8-byte aligned (one 16-byte load).
struct __attribute__((aligned(8))) EPair {
    double a, b;
};

template <int ILP>
__device__ __forceinline__ void micro_group(const XsDev &xs, const MatNuc *__restrict__ mnuc,
                                            const uint2 *h, int32_t nk, int32_t q, int32_t cnt, double e,
                                            float tb, double (&dens)[ILP], uint32_t (&ix)[ILP],
                                            double (&sc)[ILP], double (&ss)[ILP], double (&fr)[ILP],
                                            uint32_t (&pt)[ILP])
{
    uint32_t lo[ILP], hi[ILP], off[ILP], len[ILP], j[ILP];
#pragma unroll
    for (int k = 0; k < ILP; ++k) {
        const bool act = k < cnt;
        const int32_t qk = q + (act ? k : 0);  // inactive slots repeat nuclide q, in bounds
        const MatNuc mn = mnuc[qk];
        const uint2 br = h[qk];
        off[k] = mn.off;
        len[k] = mn.len;
        dens[k] = act ? mn.dens : 0.0;
        lo[k] = br.x;
        hi[k] = br.y;
        j[k] = bracket_guess(br.x, br.y, tb);
    }
    // the guess, its interval's two energies and one point on either side,
    // all nuclides' loads in flight together
    double em[ILP], eg[ILP], eg1[ILP], ep[ILP];
#pragma unroll
    for (int k = 0; k < ILP; ++k) {
        const double *g = xs.Eg + off[k];
        const EPair pr = *reinterpret_cast<const EPair *>(g + j[k]);  // j <= N - 2
        eg[k] = pr.a;
        eg1[k] = pr.b;
        em[k] = g[j[k] > 0u ? j[k] - 1u : 0u];
        ep[k] = g[j[k] + 2u < len[k] ? j[k] + 2u : len[k] - 1u];
    }
    double e0[ILP], e1[ILP];
    double2 x0[ILP], x1[ILP];
#pragma unroll
    for (int k = 0; k < ILP; ++k) {
        // i(E) = max{i : E_i <= E} clamped to [0, N-2]: j - 1, j or j + 1 when
        // those energies bracket E; else (a far guess, or the hash bin
        // computed one off at a bin edge) a walk to the defined index
        const bool dn = j[k] > 0u && e < eg[k];
        const bool up = !dn && j[k] + 2u < len[k] && e >= eg1[k];
        uint32_t i = dn ? j[k] - 1u : (up ? j[k] + 1u : j[k]);
        e0[k] = dn ? em[k] : (up ? eg1[k] : eg[k]);
        e1[k] = dn ? eg[k] : (up ? ep[k] : eg1[k]);
        if (k < cnt && ((i > 0u && e < e0[k]) || (i + 2u < len[k] && e >= e1[k]))) {
            const double *g = xs.Eg + off[k];
            while (i > 0u && e < g[i]) --i;
            while (i + 2u < len[k] && e >= g[i + 1u]) ++i;
            e0[k] = g[i];
            e1[k] = g[i + 1u];
        }
        ix[k] = i;
    }
#pragma unroll
    for (int k = 0; k < ILP; ++k) {
        x0[k] = xs.xs[off[k] + ix[k]];
        x1[k] = xs.xs[off[k] + ix[k] + 1u];
    }
#pragma unroll
    for (int k = 0; k < ILP; ++k) {
        const double f = (e - e0[k]) / (e1[k] - e0[k]);
        sc[k] = x0[k].x + f * (x1[k].x - x0[k].x);
        ss[k] = x0[k].y + f * (x1[k].y - x0[k].y);
        fr[k] = f;
        pt[k] = off[k] + ix[k];
    }
}

// The same without the interpolation fraction and table position.
template <int ILP>
__device__ __forceinline__ void micro_group(const XsDev &xs, const MatNuc *__restrict__ mnuc,
                                            const uint2 *h, int32_t nk, int32_t q, int32_t cnt, double e,
                                            float tb, double (&dens)[ILP], uint32_t (&ix)[ILP],
                                            double (&sc)[ILP], double (&ss)[ILP])
{
    double fr[ILP];
    uint32_t pt[ILP];
    micro_group<ILP>(xs, mnuc, h, nk, q, cnt, e, tb, dens, ix, sc, ss, fr, pt);
}

// Adds density * (channel x of point pt interpolated with fraction f) into
// acc[x] for the nuclides k < cnt of a group, in material order.
template <int ILP>
__device__ __forceinline__ void channel_group(const XsDev &xs, int32_t cnt, const double (&dens)[ILP],
                                              const double (&fr)[ILP], const uint32_t (&pt)[ILP],
                                              double (&acc)[MAX_CHAN])
{
    const int32_t K = xs.n_chan;
#pragma unroll
    for (int k = 0; k < ILP; ++k) {
        if (k < cnt) {
            const double *r0 = xs.xc + (size_t)pt[k] * (size_t)K;
            const double *r1 = r0 + K;
#pragma unroll
            for (int x = 0; x < MAX_CHAN; ++x)
                if (x < K) acc[x] = acc[x] + dens[k] * (r0[x] + fr[k] * (r1[x] - r0[x]));
        }
    }
}

// Hash row pointer of bin b of material m (global memory).
__device__ __forceinline__ const uint2 *hash_row(const XsDev &xs, int32_t m, int32_t b, int32_t nk)
{
    return xs.hash + xs.hash_off[m] + (uint64_t)b * (uint64_t)nk;
}

// ---------------------------------------------------------------------------
// kinematics
// ---------------------------------------------------------------------------
// Elastic scattering off a target of mass ratio A at rest, isotropic in the
// centre-of-mass frame with cosine mu: E' = E (A^2 + 2 A mu + 1)/(A + 1)^2 and
// lab cosine (1 + A mu)/sqrt(A^2 + 2 A mu + 1).
__device__ __forceinline__ void elastic_at_rest(double A, double e, double mu, double &e_out,
                                                double &mu_lab)
{
    const double q = A * A + 2.0 * A * mu + 1.0;
    e_out = e * (q / ((A + 1.0) * (A + 1.0)));
    mu_lab = (1.0 + A * mu) / sqrt(q);
}

// Turn direction (u, v, w) through polar cosine mu and azimuth phi.
__device__ __forceinline__ void turn(double &u, double &v, double &w, double mu, double phi)
{
    const double st = sqrt(fmax(0.0, 1.0 - mu * mu));
    double sp, cp;
    sincos(phi, &sp, &cp);
    double den = sqrt(fmax(0.0, 1.0 - w * w));
    double nu, nv, nw;
    if (den > 1e-10) {
        nu = mu * u + st * (u * w * cp - v * sp) / den;
        nv = mu * v + st * (v * w * cp + u * sp) / den;
        nw = mu * w - st * den * cp;
    } else {
        den = sqrt(fmax(0.0, 1.0 - v * v));
        nu = mu * u + st * (u * v * cp - w * sp) / den;
        nv = mu * v - st * den * cp;
        nw = mu * w + st * (v * w * cp + u * sp) / den;
    }
    u = nu; v = nv; w = nw;
}

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------
__device__ __forceinline__ int32_t region_material(const GeomDev &g, int32_t cell, bool inside)
{
    if (g.kind == GEOM_LATTICE) return inside ? g.pin_mat[cell] : g.mod_mat;
    if (g.kind == GEOM_SLAB) return g.layer_mat[cell];
    return g.inf_mat;
}

// Cell and cylinder sense of a point (lattice) or its layer (slab).
__device__ __forceinline__ void locate_point(const GeomDev &g, double x, double y, int32_t &cell,
                                             bool &inside)
{
    inside = false;
    cell = 0;
    if (g.kind == GEOM_LATTICE) {
        int32_t i = (int32_t)floor(x / g.pitch), j = (int32_t)floor(y / g.pitch);
        i = i < 0 ? 0 : (i > g.nx - 1 ? g.nx - 1 : i);
        j = j < 0 ? 0 : (j > g.ny - 1 ? g.ny - 1 : j);
        cell = j * g.nx + i;
        const double dx = x - ((double)i + 0.5) * g.pitch, dy = y - ((double)j + 0.5) * g.pitch;
        inside = g.pin_mat[cell] >= 0 && (dx * dx + dy * dy < g.radius * g.radius);
    } else if (g.kind == GEOM_SLAB) {
        int32_t l = 0;
        while (l < g.n_layers - 1 && x >= g.x_edges[l + 1]) ++l;
        cell = l;
    }
}

// Distance to the nearest surface bounding the particle's region and which
// one (ties resolved in the order cylinder, x, y, z).
__device__ __forceinline__ double surface_distance(const GeomDev &g, double x, double y, double z,
                                                   double u, double v, double w, int32_t cell,
                                                   bool inside, uint8_t &ev)
{
    ev = EV_COLLIDE;
    double best = INFINITY;
    if (g.kind == GEOM_INFINITE) return best;
    if (g.kind == GEOM_SLAB) {
        if (u > 0.0) { best = (g.x_edges[cell + 1] - x) / u; ev = EV_XHI; }
        else if (u < 0.0) { best = (g.x_edges[cell] - x) / u; ev = EV_XLO; }
        return best < 0.0 ? 0.0 : best;
    }
    const int32_t ci = cell % g.nx, cj = cell / g.nx;
    const double P = g.pitch;
    if (g.pin_mat[cell] >= 0) {
        const double xr = x - ((double)ci + 0.5) * P, yr = y - ((double)cj + 0.5) * P;
        const double a = u * u + v * v;
        const double k = xr * u + yr * v;
        const double c = xr * xr + yr * yr - g.radius * g.radius;
        const double disc = k * k - a * c;
        double t = INFINITY;
        if (a > 0.0) {
            if (inside) t = fmax((-k + sqrt(fmax(disc, 0.0))) / a, 0.0);
            else if (k < 0.0 && disc > 0.0) t = fmax((-k - sqrt(disc)) / a, 0.0);
        }
        if (t < best) { best = t; ev = EV_CYL; }
    }
    if (!inside) {
        if (u != 0.0) {
            const double t = fmax((u > 0.0 ? ((double)ci + 1.0) * P - x : (double)ci * P - x) / u, 0.0);
            if (t < best) { best = t; ev = u > 0.0 ? EV_XHI : EV_XLO; }
        }
        if (v != 0.0) {
            const double t = fmax((v > 0.0 ? ((double)cj + 1.0) * P - y : (double)cj * P - y) / v, 0.0);
            if (t < best) { best = t; ev = v > 0.0 ? EV_YHI : EV_YLO; }
        }
    }
    if (w != 0.0) {
        const double t = fmax((w > 0.0 ? g.z1 - z : g.z0 - z) / w, 0.0);
        if (t < best) { best = t; ev = w > 0.0 ? EV_ZHI : EV_ZLO; }
    }
    return best;
}

// ---------------------------------------------------------------------------
// wave / block helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Lane j's value (j the same in every lane) in every lane.
__device__ __forceinline__ double lane_f64(double v, int j)
{
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), j),
                            __builtin_amdgcn_readlane(__double2loint(v), j));
}

// One DPP step on a double: lane i receives the value the control selects
// (0 where the row/bank mask or the pattern gives it none).
template <int CTRL, int ROWS, int BANKS>
__device__ __forceinline__ double dpp_f64(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, BANKS, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, BANKS, false);
    return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wave, the same value in every lane: a fixed tree
// of DPP steps (quad sums, rows, then rows 0+1 and 2+3 into lane 63), read
// from lane 63.  Precondition: all 64 lanes are active (an inactive lane's
// value would be read as whatever its register holds), so callers pass 0.0
// from the lanes that contribute nothing instead of masking them off.
__device__ __forceinline__ double wave_sum(double v)
{
    v = v + dpp_f64<0xb1, 0xf, 0xf>(v);   // quad_perm 1,0,3,2
    v = v + dpp_f64<0x4e, 0xf, 0xf>(v);   // quad_perm 2,3,0,1: quad sums
    v = v + dpp_f64<0x114, 0xf, 0xe>(v);  // row_shr 4 into banks 1-3
    v = v + dpp_f64<0x118, 0xf, 0xc>(v);  // row_shr 8 into banks 2-3: row sum in lane 15 of each row
    v = v + dpp_f64<0x142, 0xa, 0xf>(v);  // row_bcast 15 into rows 1, 3
    v = v + dpp_f64<0x143, 0xc, 0xf>(v);  // row_bcast 31 into rows 2, 3: the sum in lane 63
    return lane_f64(v, 63);
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }

// The GPU hands consecutive workgroups of a launch to its 8 XCDs in turn, and
// each XCD has its own L2.  For a queue whose neighbouring entries read the
// same table lines (a sorted lookup queue), this maps workgroup b to the
// block of work it takes so that XCD_CHUNK neighbouring blocks run on one
// XCD: the launch is cut into runs of 8 XCD_CHUNK blocks, and within a run
// XCD x (b mod 8) takes blocks x XCD_CHUNK .. x XCD_CHUNK + XCD_CHUNK - 1 in
// order.  The XCDs still move through the queue together (the grid is sized
// for the longest queue, and only its first blocks have work), and blocks
// past the last whole run keep their own index.  A bijection of [0, G)
// whatever the placement; only the L2 sharing depends on it.
#ifndef MC_XCD_CHUNK
#define MC_XCD_CHUNK 4u
#endif
constexpr uint32_t XCD_CHUNK = MC_XCD_CHUNK;
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t G)
{
    constexpr uint32_t RUN = 8u * XCD_CHUNK;
    if (b >= G / RUN * RUN) return b;
    const uint32_t run = b / RUN, k = b % RUN;
    return run * RUN + (k & 7u) * XCD_CHUNK + (k >> 3);
}

}  // namespace mc

namespace mc {
// ---------------------------------------------------------------------------
// windowed multipole data (on-the-fly Doppler broadening)
// ---------------------------------------------------------------------------
constexpr int FAD_N = 32;  // terms of the rational Faddeeva series

struct MpNuc {
    uint32_t p_off, w_off, bg_off;  // first pole, window, background row
    int32_t n_windows, n_bg, pad;
    double u_lo, du;                // windows [u_lo + w du, u_lo + (w + 1) du)
};

struct MpDev {
    const MpNuc *nuc;
    const double2 *poles, *rc, *rs;  // per pole (re, im)
    const int2 *win;                 // per window [start, end) poles
    const double *bgc, *bgs;         // per window n_bg coefficients of u^-1, u^0, ...
    const int32_t *mat_off, *mat_nuc;
    const double *mat_dens, *mat_beta;  // per (material, position): density, sqrt(A / (k_B T))
    const double *fa;                // a_1 .. a_N of the Faddeeva series (fa[n - 1])
    double fL;                       // its L
    int32_t n_mat;
};

// Faddeeva function w(z) for Im z > 0 by the rational series of Weideman
// (1994): with d = L - i z and Z = (L + i z) / d,
//   w = 2 sum_{n=1..N} a_n Z^(n-1) / d^2 + pi^(-1/2) / d.
__device__ __forceinline__ void faddeeva(const MpDev &mp, double zr, double zi, double &wr, double &wi)
{
    const double L = mp.fL;
    const double dr = L + zi, di = -zr;
    const double nr = L - zi, ni = zr;
    const double dd = dr * dr + di * di;
    const double rdd = 1.0 / dd;
    const double Zr = (nr * dr + ni * di) * rdd, Zi = (ni * dr - nr * di) * rdd;
    // Horner, p = p Z + a_n with fused multiply-adds
    double pr = mp.fa[FAD_N - 1], pi_ = 0.0;
#pragma unroll 8
    for (int n = FAD_N - 2; n >= 0; --n) {
        const double tr = fma(pr, Zr, fma(-pi_, Zi, mp.fa[n]));
        const double ti = fma(pr, Zi, pi_ * Zr);
        pr = tr;
        pi_ = ti;
    }
    const double ir = dr * rdd, ii = -di * rdd;
    const double i2r = ir * ir - ii * ii, i2i = 2.0 * ir * ii;
    const double sp = 0.56418958354775628695;  // 1 / sqrt(pi)
    wr = 2.0 * (pr * i2r - pi_ * i2i) + sp * ir;
    wi = 2.0 * (pr * i2i + pi_ * i2r) + sp * ii;
}
}  // namespace mc
