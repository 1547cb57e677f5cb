/*
 * oracle.c -- plain, slow CPU oracle for the Monte Carlo transport hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library includes, links or
 * calls this file; only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg load it (through oracle/__init__.py).  It shares no code,
 * header, table or constant with the GPU path: it reads the same synthetic
 * input arrays and nothing else.
 *
 * What it computes follows the paper (Tramm et al., "Performance Portable Monte
 * Carlo Particle Transport on Intel, NVIDIA, and AMD GPUs"):
 *   - history-based tracking, one particle birth to death at a time, the mode
 *     the paper uses on CPUs (section 2, paragraph "Event-Based Parallelism";
 *     section 3);
 *   - surface tracking (ray tracing) through the geometry, delta tracking
 *     disabled (section 3);
 *   - macroscopic cross sections summed over a material's nuclides, the
 *     expensive step of the method (section 2 "Sorting"; section 4.1);
 *   - tallies scored during active batches (section 2 "Tallying"; section 4.1).
 * The paper gives no lower-level algorithm, so every other step is written
 * from its plain textbook definition; each such reading is named where it is
 * used.  Floating point is fp64 throughout, compiled with -ffp-contract=off so
 * that every expression rounds exactly as written.
 *
 * Exported functions use the prefix orc_.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* problem description (mirrored by ctypes in oracle/__init__.py)           */
/* ------------------------------------------------------------------------ */
enum { GEOM_INFINITE = 0, GEOM_LATTICE = 1, GEOM_SLAB = 2 };
enum { BC_REFLECT = 0, BC_VACUUM = 1 };
enum { SRC_POINT = 0, SRC_BOX = 1, SRC_BEAM = 2 };
enum { TALLY_ENERGY = 0, TALLY_PIN = 1, TALLY_MESH = 2, TALLY_SLAB = 3 };

/* global tally slots (each a sum over histories) */
enum {
    G_TRACK = 0,       /* sum w*d over all flights                        */
    G_COLL_EST = 1,    /* sum w/Sigma_t over collisions                   */
    G_ABSORB = 2,      /* sum w over absorptions                          */
    G_CUTOFF = 3,      /* sum w killed by the energy cutoff               */
    G_LEAK = 4,        /* sum w leaked through any vacuum face            */
    G_TRACK_ABS = 5,   /* sum w*d*Sigma_a (track-length absorption)       */
    G_NCOLL = 6,       /* number of collisions                            */
    G_NCROSS = 7,      /* number of surface crossings                     */
    G_LEAK_XHI = 8,    /* sum w leaked through the x+ face                */
    G_LEAK_XHI_UNC = 9,/* same, histories that never collided             */
    G_SPLIT = 10,      /* copies created by weight-window splitting       */
    G_ROULETTE = 11,   /* particles killed by weight-window roulette      */
    N_GLOBAL = 12
};

enum { FATE_ALIVE = 0, FATE_ABSORBED = 1, FATE_CUTOFF = 2, FATE_LEAKED = 3, FATE_LOST = 4, FATE_ROULETTE = 5 };
enum { WW_OFF = 0, WW_LINEAR = 1, WW_MLP = 2 };

typedef struct {
    /* nuclides: grid of nuclide k is E[nuc_off[k] .. nuc_off[k+1]) */
    int32_t n_nuc;
    const int64_t *nuc_off;
    const double *E, *sig_c, *sig_s, *awr;
    /* materials: nuclides mat_nuc[mat_off[m] .. mat_off[m+1]) with densities mat_dens */
    int32_t n_mat;
    const int32_t *mat_off, *mat_nuc;
    const double *mat_dens;
    /* geometry */
    int32_t geom_kind, inf_material;
    int32_t nx, ny;
    double pitch, radius, z0, z1;
    const int32_t *pin_mat;
    int32_t mod_mat;
    int32_t bc[6];
    int32_t n_layers;
    const double *x_edges;
    const int32_t *layer_mat;
    /* source */
    int32_t src_kind;
    double src_pos[3], src_box[6], src_dir[3], src_E;
    /* tally */
    int32_t tally_kind, n_ebins;
    const double *e_edges;
    int32_t mesh_dims[3];
    double mesh_box[6];
    /* physics */
    double e_cut;
    int64_t max_events;
    /* weight windows: ln I from a linear form or the importance network */
    int32_t ww_kind;
    double ww_lin[3];        /* ln I = c0 + c1 f_x + c2 f_E */
    const double *ww_mlp;    /* network parameters, oracle/mlp.py flat order */
    double ww_length;        /* feature scale L */
    double ww_kappa;         /* w_L at the source point = 1 / kappa */
    double ww_ratio;         /* w_U / w_L */
    int32_t ww_nmax;         /* most copies of one split */
    int32_t ww_depth;        /* most split generations of a copy (a copy made by g splits
                                along its line splits no further once g reaches it) */
    /* importance generation (forward estimate on an x by ln E grid) */
    int32_t imp_nx, imp_ne;
    double imp_x0, imp_x1;
    double ww_ln_lo, ww_ln_hi; /* ln I is clamped to [lo, hi] (no clamp when lo >= hi) */
    /* reaction channels: n_chan extra cross sections per grid point, channel x
     * of point j of nuclide k at chan[(nuc_off[k] + j) * n_chan + x] */
    int32_t n_chan;
    const double *chan;
} orc_problem;

/* One history: fate, final energy and weight of the source particle's own
 * copy (lineage 0); collisions, crossings, draws and path length summed over
 * the source particle and all its weight-window copies. */
typedef struct {
    int32_t fate, n_coll, n_cross, pad;
    uint64_t n_draws;
    double E_final, track, weight;
} orc_history;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11, "Parallel random        */
/* numbers: as easy as 1, 2, 3").  Written from the published definition:   */
/* ten rounds; each round multiplies words 0 and 2 by the Philox constants,  */
/* mixes the high halves with words 1/3 and the key, and the key is bumped   */
/* by the Weyl constants between rounds.                                     */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += W0; k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Draw number n of particle (seed, lineage, pid): counter = (n/2, lineage,
 * pid_lo, pid_hi), key = (seed_lo, seed_hi); the even draw takes output words
 * (1:0), the odd draw words (3:2), as a 64-bit integer x; u = ((x >> 12) + 0.5)
 * * 2^-52, exact in fp64 and strictly inside (0, 1).  (Counter layout and conversion
 * are a reading of ours; the paper does not fix them.) */
double orc_uniform(uint64_t seed, uint32_t lineage, uint64_t pid, uint64_t n)
{
    uint32_t ctr[4] = {(uint32_t)(n >> 1), lineage, (uint32_t)pid, (uint32_t)(pid >> 32)};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t o[4];
    orc_philox4x32_10(ctr, key, o);
    uint64_t x = (n & 1) ? (((uint64_t)o[3] << 32) | o[2]) : (((uint64_t)o[1] << 32) | o[0]);
    return ((double)(x >> 12) + 0.5) * (1.0 / 4503599627370496.0);
}

typedef struct {
    uint64_t seed, pid, n;
    uint32_t lineage;
} rng_stream;

static double next_u(rng_stream *s)
{
    double u = orc_uniform(s->seed, s->lineage, s->pid, s->n);
    s->n += 1;
    return u;
}

/* ------------------------------------------------------------------------ */
/* cross-section lookup: the plain definition (paper section 2 "Sorting" and */
/* section 4.1 name the macroscopic lookup as the dominant cost; the hash-   */
/* grid acceleration only speeds up reaching this same result).              */
/* ------------------------------------------------------------------------ */

/* i(E) = max{ j : E_j <= E }, clamped to [0, N-2] (a grid point itself maps to
 * its own interval; E at or above the last point maps to N-2).  Written as a
 * plain bisection for the first point strictly greater than E. */
int64_t orc_grid_index(const double *grid, int64_t n, double e)
{
    int64_t lo = 0, hi = n; /* first index with grid[idx] > e lies in [lo, hi] */
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (grid[mid] > e) hi = mid; else lo = mid + 1;
    }
    int64_t i = lo - 1;
    if (i < 0) i = 0;
    if (i > n - 2) i = n - 2;
    return i;
}

/* Microscopic cross sections of nuclide k at E by linear interpolation:
 * f = (E - E_i) / (E_{i+1} - E_i);  sigma = sigma_i + f * (sigma_{i+1} - sigma_i). */
void orc_micro_xs(const orc_problem *p, int32_t k, double e, double *sc, double *ss, int64_t *idx)
{
    const int64_t off = p->nuc_off[k];
    const int64_t n = p->nuc_off[k + 1] - off;
    const double *g = p->E + off;
    int64_t i = orc_grid_index(g, n, e);
    double f = (e - g[i]) / (g[i + 1] - g[i]);
    const double *c = p->sig_c + off, *s = p->sig_s + off;
    *sc = c[i] + f * (c[i + 1] - c[i]);
    *ss = s[i] + f * (s[i + 1] - s[i]);
    if (idx) *idx = i;
}

/* Macroscopic capture and scattering cross sections of material m at E: the
 * sums over the material's nuclides, in material order, of density times the
 * microscopic value.  Sigma_t is defined as Sigma_a + Sigma_s. */
void orc_macro_xs(const orc_problem *p, int32_t m, double e, double *Sa, double *Ss)
{
    double a = 0.0, s = 0.0;
    for (int32_t q = p->mat_off[m]; q < p->mat_off[m + 1]; ++q) {
        double sc, ss;
        orc_micro_xs(p, p->mat_nuc[q], e, &sc, &ss, NULL);
        a = a + p->mat_dens[q] * sc;
        s = s + p->mat_dens[q] * ss;
    }
    *Sa = a;
    *Ss = s;
}

/* Reaction channels (the per-nuclide reaction rates a depletion calculation
 * tallies, paper section 2 "Tallying"): each channel is tabulated on the
 * nuclide's grid and interpolated like the capture and scattering cross
 * sections, with the same index and fraction; the macroscopic value of
 * channel x is the sum over the material's nuclides, in material order, of
 * density times the microscopic value. */
#define ORC_MAX_CHAN 16

void orc_micro_channels(const orc_problem *p, int32_t k, double e, double *out)
{
    const int64_t off = p->nuc_off[k];
    const int64_t n = p->nuc_off[k + 1] - off;
    const double *g = p->E + off;
    int64_t i = orc_grid_index(g, n, e);
    double f = (e - g[i]) / (g[i + 1] - g[i]);
    const int32_t K = p->n_chan;
    const double *c0 = p->chan + (off + i) * K, *c1 = p->chan + (off + i + 1) * K;
    for (int32_t x = 0; x < K; ++x) out[x] = c0[x] + f * (c1[x] - c0[x]);
}

void orc_macro_channels(const orc_problem *p, int32_t m, double e, double *out)
{
    const int32_t K = p->n_chan;
    double micro[ORC_MAX_CHAN];
    for (int32_t x = 0; x < K; ++x) out[x] = 0.0;
    for (int32_t q = p->mat_off[m]; q < p->mat_off[m + 1]; ++q) {
        orc_micro_channels(p, p->mat_nuc[q], e, micro);
        for (int32_t x = 0; x < K; ++x) out[x] = out[x] + p->mat_dens[q] * micro[x];
    }
}

/* ------------------------------------------------------------------------ */
/* collision physics (the paper's problems are restricted here to capture    */
/* and elastic scattering, non-multiplying; the target is at rest)           */
/* ------------------------------------------------------------------------ */

/* Elastic scattering off a target of mass A at rest, isotropic in the centre
 * of mass (two-body kinematics):
 *   E'      = E (A^2 + 2 A mu + 1) / (A + 1)^2
 *   mu_lab  = (1 + A mu) / sqrt(A^2 + 2 A mu + 1)                            */
void orc_elastic(double A, double e, double mu_cm, double *e_out, double *mu_lab)
{
    double t = A * A + 2.0 * A * mu_cm + 1.0;
    *e_out = e * (t / ((A + 1.0) * (A + 1.0)));
    *mu_lab = (1.0 + A * mu_cm) / sqrt(t);
}

/* Rotate the unit direction d by polar cosine mu and azimuth phi about itself
 * (standard direction-cosine update; a second frame is used when d is within
 * 1e-10 of the z axis). */
void orc_rotate(double d[3], double mu, double phi)
{
    double u = d[0], v = d[1], w = d[2];
    double a = sqrt(fmax(0.0, 1.0 - mu * mu));
    double cp = cos(phi), sp = sin(phi);
    double b = sqrt(fmax(0.0, 1.0 - w * w));
    if (b > 1e-10) {
        d[0] = mu * u + a * (u * w * cp - v * sp) / b;
        d[1] = mu * v + a * (v * w * cp + u * sp) / b;
        d[2] = mu * w - a * b * cp;
    } else {
        b = sqrt(fmax(0.0, 1.0 - v * v));
        d[0] = mu * u + a * (u * v * cp - w * sp) / b;
        d[1] = mu * v - a * b * cp;
        d[2] = mu * w + a * (v * w * cp + u * sp) / b;
    }
}

/* ------------------------------------------------------------------------ */
/* geometry: surface tracking through constructive solid geometry           */
/* ------------------------------------------------------------------------ */
enum { S_NONE = -1, S_CYL = 0, S_XLO = 1, S_XHI = 2, S_YLO = 3, S_YHI = 4, S_ZLO = 5, S_ZHI = 6 };

typedef struct {
    double r[3], d[3];
    double E, w;
    int32_t mat;
    int32_t ci, cj, inside; /* lattice cell and cylinder sense */
    int32_t layer;          /* slab layer */
    int32_t n_coll, n_cross;
} particle;

static int32_t lattice_material(const orc_problem *p, const particle *q)
{
    if (q->inside) return p->pin_mat[q->cj * p->nx + q->ci];
    return p->mod_mat;
}

/* Locate a point: lattice cell floor(x / pitch), and inside the cell's
 * cylinder when its squared distance to the axis is below r^2. */
static void locate(const orc_problem *p, particle *q)
{
    if (p->geom_kind == GEOM_INFINITE) {
        q->mat = p->inf_material;
    } else if (p->geom_kind == GEOM_LATTICE) {
        int32_t i = (int32_t)floor(q->r[0] / p->pitch), j = (int32_t)floor(q->r[1] / p->pitch);
        if (i < 0) i = 0;
        if (i > p->nx - 1) i = p->nx - 1;
        if (j < 0) j = 0;
        if (j > p->ny - 1) j = p->ny - 1;
        q->ci = i; q->cj = j;
        double dx = q->r[0] - ((double)i + 0.5) * p->pitch;
        double dy = q->r[1] - ((double)j + 0.5) * p->pitch;
        q->inside = (p->pin_mat[j * p->nx + i] >= 0) && (dx * dx + dy * dy < p->radius * p->radius);
        q->mat = lattice_material(p, q);
    } else {
        int32_t l = 0;
        while (l < p->n_layers - 1 && q->r[0] >= p->x_edges[l + 1]) ++l;
        q->layer = l;
        q->mat = p->layer_mat[l];
    }
}

/* Distance along the direction to the nearest bounding surface of the current
 * region and that surface's id.  Ties keep the first of cylinder, x, y, z. */
static double distance_to_boundary(const orc_problem *p, const particle *q, int32_t *surf)
{
    const double INF = INFINITY;
    double x = q->r[0], y = q->r[1], z = q->r[2];
    double u = q->d[0], v = q->d[1], w = q->d[2];
    double best = INF;
    *surf = S_NONE;
    if (p->geom_kind == GEOM_INFINITE) return INF;
    if (p->geom_kind == GEOM_SLAB) {
        double t = INF; int32_t s = S_NONE;
        if (u > 0.0) { t = (p->x_edges[q->layer + 1] - x) / u; s = S_XHI; }
        else if (u < 0.0) { t = (p->x_edges[q->layer] - x) / u; s = S_XLO; }
        if (t < 0.0) t = 0.0;
        *surf = s;
        return t;
    }
    /* lattice cell (ci, cj); cylinder of radius r about the cell centre */
    double P = p->pitch;
    int32_t has_pin = p->pin_mat[q->cj * p->nx + q->ci] >= 0;
    if (has_pin) {
        double xp = x - ((double)q->ci + 0.5) * P, yp = y - ((double)q->cj + 0.5) * P;
        double a = u * u + v * v;
        double k = xp * u + yp * v;
        double c = xp * xp + yp * yp - p->radius * p->radius;
        double disc = k * k - a * c;
        double t = INF;
        if (a > 0.0) {
            if (q->inside) {
                t = (-k + sqrt(fmax(disc, 0.0))) / a;
                if (t < 0.0) t = 0.0;
            } else if (k < 0.0 && disc > 0.0) {
                t = (-k - sqrt(disc)) / a;
                if (t < 0.0) t = 0.0;
            }
        }
        if (t < best) { best = t; *surf = S_CYL; }
    }
    if (!q->inside) {
        if (u != 0.0) {
            double t = (u > 0.0) ? (((double)q->ci + 1.0) * P - x) / u : ((double)q->ci * P - x) / u;
            if (t < 0.0) t = 0.0;
            if (t < best) { best = t; *surf = (u > 0.0) ? S_XHI : S_XLO; }
        }
        if (v != 0.0) {
            double t = (v > 0.0) ? (((double)q->cj + 1.0) * P - y) / v : ((double)q->cj * P - y) / v;
            if (t < 0.0) t = 0.0;
            if (t < best) { best = t; *surf = (v > 0.0) ? S_YHI : S_YLO; }
        }
    }
    if (w != 0.0) {
        double t = (w > 0.0) ? (p->z1 - z) / w : (p->z0 - z) / w;
        if (t < 0.0) t = 0.0;
        if (t < best) { best = t; *surf = (w > 0.0) ? S_ZHI : S_ZLO; }
    }
    return best;
}

/* Outer face f (0..5 = x-, x+, y-, y+, z-, z+): reflect (flip the normal
 * component, place the point exactly on the face) or leak.  Returns 1 when the
 * particle leaked. */
static int outer_face(const orc_problem *p, particle *q, int f, double face)
{
    int axis = f / 2;
    if (p->bc[f] == BC_VACUUM) return 1;
    q->d[axis] = -q->d[axis];
    q->r[axis] = face;
    return 0;
}

/* Cross surface s; returns 1 when the particle leaked. */
static int cross_surface(const orc_problem *p, particle *q, int32_t s)
{
    q->n_cross += 1;
    if (p->geom_kind == GEOM_SLAB) {
        if (s == S_XHI) {
            if (q->layer == p->n_layers - 1) return outer_face(p, q, 1, p->x_edges[p->n_layers]);
            q->layer += 1;
            q->r[0] = p->x_edges[q->layer];
        } else {
            if (q->layer == 0) return outer_face(p, q, 0, p->x_edges[0]);
            q->r[0] = p->x_edges[q->layer];
            q->layer -= 1;
        }
        q->mat = p->layer_mat[q->layer];
        return 0;
    }
    double P = p->pitch;
    switch (s) {
    case S_CYL:
        q->inside = !q->inside;
        break;
    case S_XHI:
        if (q->ci == p->nx - 1) return outer_face(p, q, 1, (double)p->nx * P);
        q->ci += 1; q->r[0] = (double)q->ci * P;
        break;
    case S_XLO:
        if (q->ci == 0) return outer_face(p, q, 0, 0.0);
        q->r[0] = (double)q->ci * P; q->ci -= 1;
        break;
    case S_YHI:
        if (q->cj == p->ny - 1) return outer_face(p, q, 3, (double)p->ny * P);
        q->cj += 1; q->r[1] = (double)q->cj * P;
        break;
    case S_YLO:
        if (q->cj == 0) return outer_face(p, q, 2, 0.0);
        q->r[1] = (double)q->cj * P; q->cj -= 1;
        break;
    case S_ZHI:
        return outer_face(p, q, 5, p->z1);
    case S_ZLO:
        return outer_face(p, q, 4, p->z0);
    default:
        break;
    }
    q->mat = lattice_material(p, q);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* tallies                                                                   */
/* ------------------------------------------------------------------------ */
static int64_t tally_bins(const orc_problem *p)
{
    switch (p->tally_kind) {
    case TALLY_ENERGY: return p->n_ebins;
    case TALLY_PIN: return (int64_t)p->nx * p->ny;
    case TALLY_MESH: return (int64_t)p->mesh_dims[0] * p->mesh_dims[1] * p->mesh_dims[2];
    case TALLY_SLAB: return p->n_layers;
    }
    return 0;
}

/* energy bins are [e_b, e_{b+1}); the top edge belongs to the last bin */
static int64_t energy_bin(const orc_problem *p, double e)
{
    int64_t n = p->n_ebins;
    if (e < p->e_edges[0] || e > p->e_edges[n]) return -1;
    if (e == p->e_edges[n]) return n - 1;
    int64_t b = 0;
    while (b < n - 1 && e >= p->e_edges[b + 1]) ++b;
    return b;
}

static int64_t mesh_cell(const orc_problem *p, const double r[3])
{
    int64_t idx[3];
    for (int a = 0; a < 3; ++a) {
        double lo = p->mesh_box[2 * a], hi = p->mesh_box[2 * a + 1];
        if (r[a] < lo || r[a] > hi) return -1;
        int64_t c = (int64_t)floor((r[a] - lo) / (hi - lo) * p->mesh_dims[a]);
        if (c > p->mesh_dims[a] - 1) c = p->mesh_dims[a] - 1;
        idx[a] = c;
    }
    return (idx[2] * p->mesh_dims[1] + idx[1]) * p->mesh_dims[0] + idx[0];
}

/* bin of a point event (collision) */
static int64_t point_bin(const orc_problem *p, const particle *q)
{
    switch (p->tally_kind) {
    case TALLY_ENERGY: return energy_bin(p, q->E);
    case TALLY_PIN: return q->inside ? (int64_t)q->cj * p->nx + q->ci : -1;
    case TALLY_MESH: return mesh_cell(p, q->r);
    case TALLY_SLAB: return q->layer;
    }
    return -1;
}

static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* Track-length score w * (length of the flight inside each bin).  For the
 * mesh: the flight from r0 over length d is cut at every mesh plane it
 * crosses; each piece is scored into the cell holding its midpoint. */
static void score_flight(const orc_problem *p, const particle *q, const double r0[3], double d,
                         double *tl)
{
    if (p->tally_kind != TALLY_MESH) {
        int64_t b = point_bin(p, q);
        if (b >= 0) tl[b] += q->w * d;
        return;
    }
    double cuts[4096];
    int nc = 0;
    cuts[nc++] = 0.0;
    for (int a = 0; a < 3; ++a) {
        double da = q->d[a];
        if (da == 0.0) continue;
        double lo = p->mesh_box[2 * a], hi = p->mesh_box[2 * a + 1];
        double h = (hi - lo) / p->mesh_dims[a];
        for (int32_t k = 0; k <= p->mesh_dims[a]; ++k) {
            double t = (lo + k * h - r0[a]) / da;
            if (t > 0.0 && t < d && nc < 4095) cuts[nc++] = t;
        }
    }
    qsort(cuts, nc, sizeof(double), cmp_double);
    cuts[nc++] = d;
    for (int k = 0; k + 1 < nc; ++k) {
        double len = cuts[k + 1] - cuts[k];
        if (len <= 0.0) continue;
        double tm = 0.5 * (cuts[k] + cuts[k + 1]);
        double pm[3] = {r0[0] + tm * q->d[0], r0[1] + tm * q->d[1], r0[2] + tm * q->d[2]};
        int64_t b = mesh_cell(p, pm);
        if (b >= 0) tl[b] += q->w * len;
    }
}

/* ------------------------------------------------------------------------ */
/* importance network (forward only, FP64 with BF16 rounding points; the     */
/* same network as oracle/mlp.py)                                            */
/* ------------------------------------------------------------------------ */
/* Nearest BF16 value of x (ties to even), via FP32. */
double orc_bf16(double x)
{
    float f = (float)x;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return x; /* NaN */
    u = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

static double silu(double z) { return z / (1.0 + exp(-z)); }

/* ln I of features f[4]: z1 = bf16(f) W1 + b1, h1 = bf16(silu(z1)),
 * z2 = h1 W2 + b2, h2 = silu(z2), y = h2 w3 + b3 (W1, W2, w3 as BF16). */
double orc_mlp_forward(const double *prm, const double f[4])
{
    const double *W1 = prm, *b1 = prm + 256, *W2 = prm + 320, *b2 = prm + 4416, *w3 = prm + 4480;
    const double b3 = prm[4544];
    double h1[64], y = 0.0;
    double fr[4];
    for (int k = 0; k < 4; ++k) fr[k] = orc_bf16(f[k]);
    for (int j = 0; j < 64; ++j) {
        double z = 0.0;
        for (int k = 0; k < 4; ++k) z = z + fr[k] * orc_bf16(W1[k * 64 + j]);
        h1[j] = orc_bf16(silu(z + b1[j]));
    }
    for (int j = 0; j < 64; ++j) {
        double z = 0.0;
        for (int k = 0; k < 64; ++k) z = z + h1[k] * orc_bf16(W2[k * 64 + j]);
        y = y + silu(z + b2[j]) * orc_bf16(w3[j]);
    }
    return y + b3;
}

/* importance features: (x/L, clip(y/L), clip(z/L), (ln E - ln 1e-5)/ln(2e7/1e-5)) */
static void ww_features(const orc_problem *p, const double r[3], double E, double f[4])
{
    const double L = p->ww_length;
    f[0] = r[0] / L;
    f[1] = fmin(1.0, fmax(-1.0, r[1] / L));
    f[2] = fmin(1.0, fmax(-1.0, r[2] / L));
    f[3] = (log(E) - log(1e-5)) / log(2e7 / 1e-5);
}

static double ln_importance(const orc_problem *p, const double r[3], double E)
{
    double f[4], v;
    ww_features(p, r, E, f);
    if (p->ww_kind == WW_LINEAR) v = p->ww_lin[0] + p->ww_lin[1] * f[0] + p->ww_lin[2] * f[3];
    else v = orc_mlp_forward(p->ww_mlp, f);
    /* a map is trusted over the span it was fitted on */
    if (p->ww_ln_lo < p->ww_ln_hi) v = fmin(fmax(v, p->ww_ln_lo), p->ww_ln_hi);
    return v;
}

/* Lineage of split copy k (1..n-1) of split number s of a particle of
 * lineage a: a hash of the three (MurmurHash3's 32-bit finaliser); never 0,
 * which is the primary particles' lineage. */
uint32_t orc_child_lineage(uint32_t a, uint32_t s, uint32_t k)
{
    uint32_t h = a * 0x9E3779B1u;
    h ^= (s + 0x7F4A7C15u) * 0x85EBCA77u;
    h ^= (k + 1u) * 0xC2B2AE3Du;
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h ? h : 1u;
}

/* ------------------------------------------------------------------------ */
/* one history, birth to death (paper section 2: history-based mode)        */
/* ------------------------------------------------------------------------ */
static void sample_source(const orc_problem *p, particle *q, rng_stream *rs)
{
    memset(q, 0, sizeof(*q));
    q->E = p->src_E;
    q->w = 1.0;
    if (p->src_kind == SRC_BEAM) {
        for (int a = 0; a < 3; ++a) { q->r[a] = p->src_pos[a]; q->d[a] = p->src_dir[a]; }
    } else {
        if (p->src_kind == SRC_BOX) {
            for (int a = 0; a < 3; ++a) {
                double lo = p->src_box[2 * a], hi = p->src_box[2 * a + 1];
                q->r[a] = lo + (hi - lo) * next_u(rs);
            }
        } else {
            for (int a = 0; a < 3; ++a) q->r[a] = p->src_pos[a];
        }
        /* isotropic: mu = 2 xi - 1 is the z cosine, phi = 2 pi xi the azimuth */
        double mu = 2.0 * next_u(rs) - 1.0;
        double phi = 2.0 * M_PI * next_u(rs);
        double s = sqrt(fmax(0.0, 1.0 - mu * mu));
        q->d[0] = s * cos(phi);
        q->d[1] = s * sin(phi);
        q->d[2] = mu;
    }
    locate(p, q);
}

#define IMP_MAX_WORDS 64  /* importance grid of at most 4096 cells */
#define WW_MAX_DEPTH 64

/* A particle copy: its state, its random stream and the importance cells it
 * (or the particle it was split from) has entered. */
typedef struct {
    particle q;
    rng_stream rs;
    uint32_t splits;     /* split events of this copy (numbers its children) */
    uint32_t gen;        /* splits along the line from the source particle to this copy */
    uint64_t seen[IMP_MAX_WORDS];
} copy_state;

/* n - 1 identical pending copies of a split, handed out last-in first-out */
typedef struct {
    copy_state proto;    /* state at the split (weight already divided) */
    uint32_t lineage, split_no, next_k, n;
} split_record;

typedef struct {
    double *tl, *coll, *glob, *imp; /* imp: num[nc], den[nc], cnt[nc] */
    double *rr;                     /* reaction rates [n_mat][n_chan] (track length) */
    double *ns;                     /* test statistics per target nuclide [n_nuc][2]:
                                       scatterings, sum of ln(E / E') (nullable) */
} scores;

static int64_t imp_cell(const orc_problem *p, double x, double E)
{
    int64_t ix = (int64_t)floor((x - p->imp_x0) / (p->imp_x1 - p->imp_x0) * p->imp_nx);
    int64_t ie = (int64_t)floor((log(E) - log(1e-5)) / log(2e7 / 1e-5) * p->imp_ne);
    if (ix < 0) ix = 0;
    if (ix > p->imp_nx - 1) ix = p->imp_nx - 1;
    if (ie < 0) ie = 0;
    if (ie > p->imp_ne - 1) ie = p->imp_ne - 1;
    return ie * p->imp_nx + ix;
}

/* Mark the importance cells of x-bins between x0 and x1 at energy E as
 * entered; the weight entering a cell counts the first time only. */
static void imp_enter(const orc_problem *p, copy_state *c, double x0, double x1, double E, double *den)
{
    if (!p->imp_nx) return;
    int64_t a = imp_cell(p, x0, E), b = imp_cell(p, x1, E);
    if (a > b) { int64_t t = a; a = b; b = t; }
    for (int64_t g = a; g <= b; ++g) {
        uint64_t bit = 1ull << (g & 63);
        if (!(c->seen[g >> 6] & bit)) {
            c->seen[g >> 6] |= bit;
            den[g] += c->q.w;
        }
    }
}

/* A detector score w credits every cell the copy's line has entered. */
static void imp_credit(const orc_problem *p, const copy_state *c, double w, double *num, double *cnt)
{
    if (!p->imp_nx) return;
    int64_t nc = (int64_t)p->imp_nx * p->imp_ne;
    for (int64_t g = 0; g < nc; ++g)
        if (c->seen[g >> 6] & (1ull << (g & 63))) {
            num[g] += w;
            cnt[g] += 1.0;
        }
}

/* Weight-window game after a collision or a crossing.  Window of the point:
 * w_L = exp(ln I_src - ln I) / kappa, w_U = ratio * w_L, survival weight
 * w_S = (w_L + w_U) / 2.  Above w_U: split into n = min(n_max, ceil(w / w_U))
 * copies of weight w / n (copy 0 goes on, n - 1 are pushed); below w_L:
 * roulette, surviving with probability w / w_S at weight w_S (one draw).
 * Returns 1 when the particle was killed. */
static int weight_window(const orc_problem *p, copy_state *c, double ln_src, split_record *stack, int *depth,
                         double *glob)
{
    const double lw = exp(ln_src - ln_importance(p, c->q.r, c->q.E)) / p->ww_kappa;
    const double uw = p->ww_ratio * lw;
    const double sw = 0.5 * (lw + uw);
    const double w = c->q.w;
    if (w > uw) {
        int32_t n = (int32_t)ceil(w / uw);
        if (n > p->ww_nmax) n = p->ww_nmax;
        if (n >= 2 && c->gen < (uint32_t)p->ww_depth) {
            c->gen += 1; /* the copy that goes on and its n - 1 siblings */
            c->q.w = w / (double)n;
            split_record *r = &stack[(*depth)++];
            r->proto = *c;
            r->lineage = c->rs.lineage;
            r->split_no = c->splits;
            r->next_k = 1;
            r->n = (uint32_t)n;
            c->splits += 1;
            glob[G_SPLIT] += (double)(n - 1);
        }
        return 0;
    }
    if (w < lw) {
        if (next_u(&c->rs) < w / sw) {
            c->q.w = sw;
            return 0;
        }
        glob[G_ROULETTE] += 1.0;
        return 1;
    }
    return 0;
}

static void track_history(const orc_problem *p, uint64_t seed, uint64_t pid, scores sc, double ln_src,
                          orc_history *h)
{
    double *tl = sc.tl, *coll = sc.coll, *glob = sc.glob;
    const int64_t ncell = (int64_t)p->imp_nx * p->imp_ne;
    double *num = sc.imp, *den = sc.imp ? sc.imp + ncell : NULL, *cnt = sc.imp ? sc.imp + 2 * ncell : NULL;
    split_record stack[WW_MAX_DEPTH];
    int depth = 0;
    copy_state c;
    memset(&c, 0, sizeof c);
    c.rs.seed = seed;
    c.rs.pid = pid;
    sample_source(p, &c.q, &c.rs);
    if (den) imp_enter(p, &c, c.q.r[0], c.q.r[0], c.q.E, den);
    int fate = FATE_ALIVE, fate0 = FATE_ALIVE;
    double E0 = 0.0, w0 = 0.0;
    double track = 0.0;
    int64_t n_coll = 0, n_cross = 0;
    uint64_t n_draws = 0;
    for (;;) {
        if ((int64_t)c.q.n_coll + c.q.n_cross >= p->max_events) { fate = FATE_LOST; goto dead; }
        double Sa, Ss;
        orc_macro_xs(p, c.q.mat, c.q.E, &Sa, &Ss);
        double St = Sa + Ss;
        double Sx[ORC_MAX_CHAN];
        if (sc.rr) orc_macro_channels(p, c.q.mat, c.q.E, Sx);
        /* distance to collision: -ln(xi) / Sigma_t */
        double dc = -log(next_u(&c.rs)) / St;
        int32_t surf;
        double db = distance_to_boundary(p, &c.q, &surf);
        double d = (db < dc) ? db : dc;
        double r0[3] = {c.q.r[0], c.q.r[1], c.q.r[2]};
        for (int a = 0; a < 3; ++a) c.q.r[a] = c.q.r[a] + d * c.q.d[a];
        score_flight(p, &c.q, r0, d, tl);
        glob[G_TRACK] += c.q.w * d;
        glob[G_TRACK_ABS] += c.q.w * d * Sa;
        if (sc.rr) {
            /* track-length reaction rates: weight * path * Sigma_x in the flight's material */
            double *r = sc.rr + (int64_t)c.q.mat * p->n_chan;
            for (int32_t x = 0; x < p->n_chan; ++x) r[x] += c.q.w * d * Sx[x];
        }
        track += d;
        if (den) imp_enter(p, &c, r0[0], c.q.r[0], c.q.E, den);
        if (db < dc) {
            glob[G_NCROSS] += 1.0;
            int face_xhi = (p->geom_kind != GEOM_INFINITE) && (surf == S_XHI) &&
                           ((p->geom_kind == GEOM_SLAB) ? (c.q.layer == p->n_layers - 1) : (c.q.ci == p->nx - 1));
            if (cross_surface(p, &c.q, surf)) {
                fate = FATE_LEAKED;
                glob[G_LEAK] += c.q.w;
                if (face_xhi) {
                    glob[G_LEAK_XHI] += c.q.w;
                    if (c.q.n_coll == 0) glob[G_LEAK_XHI_UNC] += c.q.w;
                    if (num) imp_credit(p, &c, c.q.w, num, cnt);
                }
                goto dead;
            }
            if (p->ww_kind && weight_window(p, &c, ln_src, stack, &depth, glob)) {
                fate = FATE_ROULETTE;
                goto dead;
            }
            continue;
        }
        /* collision */
        c.q.n_coll += 1;
        glob[G_NCOLL] += 1.0;
        {
            int64_t b = point_bin(p, &c.q);
            if (b >= 0) coll[b] += c.q.w / St;
            glob[G_COLL_EST] += c.q.w / St;
        }
        /* analog absorption: absorbed when xi * Sigma_t < Sigma_a */
        if (next_u(&c.rs) * St < Sa) {
            glob[G_ABSORB] += c.q.w;
            fate = FATE_ABSORBED;
            goto dead;
        }
        {
            /* target nuclide: the first, in material order, whose running
             * sum of density * sigma_s reaches xi * Sigma_s */
            double target = next_u(&c.rs) * Ss;
            double cum = 0.0;
            int32_t nuc = -1;
            for (int32_t qq = p->mat_off[c.q.mat]; qq < p->mat_off[c.q.mat + 1]; ++qq) {
                double sc_, ss_;
                orc_micro_xs(p, p->mat_nuc[qq], c.q.E, &sc_, &ss_, NULL);
                double term = p->mat_dens[qq] * ss_;
                cum = cum + term;
                if (term > 0.0) nuc = p->mat_nuc[qq];
                if (cum >= target && term > 0.0) break;
            }
            if (nuc < 0) {
                /* no nuclide scatters although the particle was not captured:
                 * Sigma_s = 0 and Sigma_a = 0 at once; the history cannot go on */
                fate = FATE_LOST;
                goto dead;
            }
            double mu_cm = 2.0 * next_u(&c.rs) - 1.0;
            double phi = 2.0 * M_PI * next_u(&c.rs);
            double e_out, mu_lab;
            orc_elastic(p->awr[nuc], c.q.E, mu_cm, &e_out, &mu_lab);
            orc_rotate(c.q.d, mu_lab, phi);
            if (sc.ns) {
                sc.ns[2 * nuc] += 1.0;
                sc.ns[2 * nuc + 1] += log(c.q.E / e_out);
            }
            c.q.E = e_out;
        }
        if (c.q.E < p->e_cut) {
            glob[G_CUTOFF] += c.q.w;
            fate = FATE_CUTOFF;
            goto dead;
        }
        if (den) imp_enter(p, &c, c.q.r[0], c.q.r[0], c.q.E, den);
        if (p->ww_kind && weight_window(p, &c, ln_src, stack, &depth, glob)) {
            fate = FATE_ROULETTE;
            goto dead;
        }
        continue;
    dead:
        n_coll += c.q.n_coll;
        n_cross += c.q.n_cross;
        n_draws += c.rs.n;
        if (c.rs.lineage == 0) {
            /* the source particle's own copy (it keeps lineage 0 through its
             * splits) ends first: its fate, energy and weight are the record's */
            fate0 = fate;
            E0 = c.q.E;
            w0 = c.q.w;
        }
        if (depth == 0) break;
        {
            /* next pending copy: fresh stream of its own lineage */
            split_record *r = &stack[depth - 1];
            const uint32_t k = r->next_k++;
            c = r->proto;
            c.rs.lineage = orc_child_lineage(r->lineage, r->split_no, k);
            c.rs.n = 0;
            c.splits = 0;
            c.q.n_coll = r->proto.q.n_coll;
            c.q.n_cross = r->proto.q.n_cross;
            n_coll -= c.q.n_coll;   /* the copy's counts continue from its parent's */
            n_cross -= c.q.n_cross;
            if (r->next_k >= r->n) --depth;
            fate = FATE_ALIVE;
        }
    }
    if (h) {
        h->fate = fate0;
        h->n_coll = (int32_t)n_coll;
        h->n_cross = (int32_t)n_cross;
        h->n_draws = n_draws;
        h->E_final = E0;
        h->track = track;
        h->weight = w0;
    }
}

static int64_t imp_cells(const orc_problem *p) { return (int64_t)p->imp_nx * p->imp_ne; }

/* ln I at the source point (E0, the source position or the box centre) */
double orc_ln_importance_source(const orc_problem *p)
{
    double r[3];
    for (int a = 0; a < 3; ++a)
        r[a] = (p->src_kind == SRC_BOX) ? 0.5 * (p->src_box[2 * a] + p->src_box[2 * a + 1]) : p->src_pos[a];
    return ln_importance(p, r, p->src_E);
}

/* Run histories [first_pid, first_pid + n) and add their raw (un-normalised)
 * scores into tl[n_bins], coll[n_bins], glob[N_GLOBAL], when the importance
 * grid is on imp[3 * cells] (numerators, weights entered, score counts), and
 * when the problem has reaction channels and rr is given rr[n_mat * n_chan].
 * The pids are split into at most 64 contiguous blocks, each tracked in pid
 * order by one thread and summed in block order, so the result does not
 * depend on the thread count.  hist (nullable) receives one record per pid. */
static int run_blocks(const orc_problem *p, uint64_t seed, uint64_t first_pid, uint64_t n, double *tl,
                      double *coll, double *glob, double *imp, double *rr, double *ns, orc_history *hist,
                      int n_threads)
{
    int64_t nb = tally_bins(p);
    int64_t ni = imp ? 3 * imp_cells(p) : 0;
    if (p->n_chan < 0 || p->n_chan > ORC_MAX_CHAN) return -2;
    int64_t nr = (rr && p->n_chan > 0) ? (int64_t)p->n_mat * p->n_chan : 0;
    if (imp_cells(p) > 64 * IMP_MAX_WORDS) return -2;
    if (p->ww_kind && (p->ww_depth > WW_MAX_DEPTH || p->ww_depth < 0)) return -2;
    int64_t n_blocks = n < 64 ? (int64_t)n : 64;
    if (n_blocks == 0) return 0;
    int64_t nn = ns ? 2 * (int64_t)p->n_nuc : 0;
    int64_t stride = nb * 2 + N_GLOBAL + ni + nr + nn;
    double *part = (double *)calloc((size_t)(n_blocks * stride), sizeof(double));
    if (!part) return -1;
    const double ln_src = p->ww_kind ? orc_ln_importance_source(p) : 0.0;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t b = 0; b < n_blocks; ++b) {
        uint64_t lo = (uint64_t)b * n / (uint64_t)n_blocks;
        uint64_t hi = (uint64_t)(b + 1) * n / (uint64_t)n_blocks;
        double *t = part + b * stride;
        scores sc = {t, t + nb, t + 2 * nb, imp ? t + 2 * nb + N_GLOBAL : NULL,
                     nr ? t + 2 * nb + N_GLOBAL + ni : NULL, nn ? t + 2 * nb + N_GLOBAL + ni + nr : NULL};
        for (uint64_t i = lo; i < hi; ++i) track_history(p, seed, first_pid + i, sc, ln_src, hist ? hist + i : NULL);
    }
    for (int64_t b = 0; b < n_blocks; ++b) {
        const double *t = part + b * stride;
        for (int64_t k = 0; k < nb; ++k) { tl[k] += t[k]; coll[k] += t[nb + k]; }
        for (int k = 0; k < N_GLOBAL; ++k) glob[k] += t[2 * nb + k];
        for (int64_t k = 0; k < ni; ++k) imp[k] += t[2 * nb + N_GLOBAL + k];
        for (int64_t k = 0; k < nr; ++k) rr[k] += t[2 * nb + N_GLOBAL + ni + k];
        for (int64_t k = 0; k < nn; ++k) ns[k] += t[2 * nb + N_GLOBAL + ni + nr + k];
    }
    free(part);
    return 0;
}

int orc_run(const orc_problem *p, uint64_t seed, uint64_t first_pid, uint64_t n, double *tl,
            double *coll, double *glob, double *imp, double *rr, orc_history *hist, int n_threads)
{
    return run_blocks(p, seed, first_pid, n, tl, coll, glob, imp, rr, NULL, hist, n_threads);
}

/* Test statistics of the collision's target selection and kinematics: the
 * same run as orc_run (scores discarded), adding per target nuclide k the
 * number of scatterings ns[2k] and the sum of their lethargy gains
 * ln(E / E') into ns[2k + 1]. */
int orc_run_scatter_stats(const orc_problem *p, uint64_t seed, uint64_t first_pid, uint64_t n, double *ns,
                          int n_threads)
{
    int64_t nb = tally_bins(p);
    double *tl = (double *)calloc((size_t)(2 * nb + N_GLOBAL + 1), sizeof(double));
    if (!tl) return -1;
    int rc = run_blocks(p, seed, first_pid, n, tl, tl + nb, tl + 2 * nb, NULL, NULL, ns, NULL, n_threads);
    free(tl);
    return rc;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Vector forms of the two lookups above, for the tests (plain loops). */
void orc_micro_xs_many(const orc_problem *p, int32_t k, int64_t n, const double *e, int64_t *idx,
                       double *sc, double *ss)
{
    for (int64_t i = 0; i < n; ++i) orc_micro_xs(p, k, e[i], sc + i, ss + i, idx + i);
}

void orc_macro_channels_many(const orc_problem *p, int64_t n, const int32_t *mat, const double *e,
                             double *out)
{
    for (int64_t i = 0; i < n; ++i) orc_macro_channels(p, mat[i], e[i], out + i * p->n_chan);
}

void orc_macro_xs_many(const orc_problem *p, int64_t n, const int32_t *mat, const double *e, double *Sa,
                       double *Ss)
{
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (int64_t i = 0; i < n; ++i) orc_macro_xs(p, mat[i], e[i], Sa + i, Ss + i);
}

/* ------------------------------------------------------------------------ */
/* Windowed multipole cross sections with Doppler broadening on the fly      */
/* (the compute-bound alternative to tabulated data the paper points to in   */
/* section 4.1; Josey, Forget and Smith, J. Comput. Phys. 2016).  In u =     */
/* sqrt(E) a nuclide's cross section is a sum over poles p_j (Im p_j < 0)   */
/* with residues r_j, plus a smooth background:                              */
/*   sigma_x(E, T) = (1/E) sum_j Re[ r_x,j c_j(u) ] + sum_n b_x,n u^(n-1)     */
/*   c_j(u) = sqrt(pi) beta w(beta (u - p_j)),  beta = sqrt(A / (k_B T)),     */
/* w the Faddeeva function; as T -> 0, c_j -> i / (u - p_j).  Only the poles */
/* of the window holding u enter (the windows split [u_lo, u_hi] evenly).    */
/* ------------------------------------------------------------------------ */

/* Faddeeva function w(z) = exp(-z^2) erfc(-i z) for Im z > 0 by Weideman's  */
/* rational series (SIAM J. Numer. Anal. 31, 1994): with L = (N / sqrt 2)^(1/2)*/
/* and Z = (L + i z) / (L - i z),                                            */
/*   w(z) = 2 sum_{n=1..N} a_n Z^(n-1) / (L - i z)^2 + pi^(-1/2) / (L - i z), */
/* a_n the cosine coefficients of f(t) = exp(-t^2) (L^2 + t^2) on the map     */
/* t = L tan(theta / 2), sampled at theta_k = k pi / M, M = 2N.              */
#define ORC_WN 32
static double orc_wa[ORC_WN + 1], orc_wL = 0.0;

void orc_faddeeva_init(void)
{
    const int N = ORC_WN, M = 2 * N;
    const double L = sqrt(sqrt((double)N * (double)N / 2.0));
    for (int n = 1; n <= N; ++n) {
        double s = 0.0;
        for (int k = -M + 1; k <= M - 1; ++k) {
            const double th = (double)k * M_PI / (double)M;
            const double t = L * tan(th / 2.0);
            const double f = exp(-t * t) * (L * L + t * t);
            s += f * cos(M_PI * (double)n * (double)k / (double)M);
        }
        orc_wa[n] = s / (2.0 * (double)M);
    }
    orc_wL = L;
}

void orc_faddeeva(double zr, double zi, double *wr, double *wi)
{
    /* the series as written, in complex arithmetic: powers Z^(n-1) built up
     * from n = 1 and the terms added in that order */
    const double complex z = CMPLX(zr, zi);
    const double complex d = orc_wL - I * z;          /* L - i z */
    const double complex Z = (orc_wL + I * z) / d;    /* (L + i z) / (L - i z) */
    double complex s = 0.0, Zp = 1.0;                 /* Zp = Z^(n-1) */
    for (int n = 1; n <= ORC_WN; ++n) {
        s = s + orc_wa[n] * Zp;
        Zp = Zp * Z;
    }
    const double complex w = 2.0 * s / (d * d) + (1.0 / sqrt(M_PI)) / d;
    *wr = creal(w);
    *wi = cimag(w);
}

/* Weideman's constants (L and a_1..a_N) for the tests' rounding bound. */
void orc_faddeeva_coeffs(double *L, double *a)
{
    *L = orc_wL;
    for (int n = 1; n <= ORC_WN; ++n) a[n - 1] = orc_wa[n];
}

typedef struct {
    int32_t n_poles, n_windows, n_bg, pad;
    double u_lo, u_hi;
    const double *poles;  /* [n_poles][2] (re, im) */
    const double *res_c;  /* [n_poles][2] */
    const double *res_s;  /* [n_poles][2] */
    const int32_t *win;   /* [n_windows][2] pole range [start, end) */
    const double *bg_c;   /* [n_windows][n_bg] */
    const double *bg_s;
} orc_mp_nuclide;

#define ORC_KB 8.617333262e-5 /* Boltzmann constant, eV / K */

/* Microscopic capture and scattering cross sections of a multipole nuclide of
 * mass ratio A at E (eV) and temperature T (K, > 0). */
void orc_mp_micro(const orc_mp_nuclide *nd, double A, double T, double e, double *sc, double *ss)
{
    const double u = sqrt(e);
    const double beta = sqrt(A / (ORC_KB * T));
    const double du = (nd->u_hi - nd->u_lo) / (double)nd->n_windows;
    int32_t w = (int32_t)floor((u - nd->u_lo) / du);
    if (w < 0) w = 0;
    if (w > nd->n_windows - 1) w = nd->n_windows - 1;
    double c = 0.0, s = 0.0;
    for (int32_t j = nd->win[2 * w]; j < nd->win[2 * w + 1]; ++j) {
        const double complex pole = CMPLX(nd->poles[2 * j], nd->poles[2 * j + 1]);
        const double complex zz = beta * (u - pole);
        double wr, wi;
        orc_faddeeva(creal(zz), cimag(zz), &wr, &wi);
        /* c_j = sqrt(pi) beta w(beta (u - p_j)) */
        const double complex cj = sqrt(M_PI) * beta * CMPLX(wr, wi);
        c = c + creal(CMPLX(nd->res_c[2 * j], nd->res_c[2 * j + 1]) * cj);
        s = s + creal(CMPLX(nd->res_s[2 * j], nd->res_s[2 * j + 1]) * cj);
    }
    c = c / e;
    s = s / e;
    /* background: sum_n b_n u^(n-1) */
    double up = 1.0 / u;
    for (int32_t n = 0; n < nd->n_bg; ++n) {
        c += nd->bg_c[w * nd->n_bg + n] * up;
        s += nd->bg_s[w * nd->n_bg + n] * up;
        up *= u;
    }
    *sc = c;
    *ss = s;
}

/* Macroscopic values of a material (nuclides ids[0..nk), densities dens) at
 * temperature T: sums in material order. */
void orc_mp_macro_many(const orc_mp_nuclide *nucs, const double *awr, int32_t nk, const int32_t *ids,
                       const double *dens, double T, int64_t n, const double *e, double *Sa, double *Ss)
{
    for (int64_t i = 0; i < n; ++i) {
        double a = 0.0, s = 0.0;
        for (int32_t q = 0; q < nk; ++q) {
            double sc, ss;
            orc_mp_micro(&nucs[ids[q]], awr[ids[q]], T, e[i], &sc, &ss);
            a = a + dens[q] * sc;
            s = s + dens[q] * ss;
        }
        Sa[i] = a;
        Ss[i] = s;
    }
}

void orc_faddeeva_many(int64_t n, const double *zr, const double *zi, double *wr, double *wi)
{
    for (int64_t i = 0; i < n; ++i) orc_faddeeva(zr[i], zi[i], wr + i, wi + i);
}
