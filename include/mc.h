/*
 * mc.h -- C ABI of the MI355X Monte Carlo transport hot path (libmc.so).
 *
 * The library runs the event-based tracking loop of continuous-energy,
 * fixed-source, non-multiplying neutral-particle transport (capture and
 * elastic scattering) on one AMD Instinct MI355X (gfx950), the GPU mode of the
 * paper "Performance Portable Monte Carlo Particle Transport on Intel, NVIDIA,
 * and AMD GPUs" (Tramm et al.): particles in flight are processed one event
 * type at a time over the whole bank (section 2, "Event-Based Parallelism"),
 * the cross-section lookup queue is sorted by material and energy first
 * (section 2, "Sorting"), the number of particles in flight is capped and
 * refilled from the batch (section 2, "In-Flight Particles"), and tallies are
 * scored during active batches (section 2, "Tallying"; section 4.1).
 *
 * Conventions for every entry point:
 *   - Return value: MC_OK (0) or a negative mc_status.  No C++ exception
 *     crosses the ABI.  mc_last_error() gives the reason as text.
 *   - Host arrays passed to mc_init_* are read during the call and deep-copied
 *     to device memory; the caller keeps ownership.
 *   - Pointers documented as "device" must point to device memory of the
 *     context's GPU (for example a torch tensor's data_ptr()); the library
 *     neither frees nor retains them beyond the call.
 *   - All GPU work is enqueued on the context's HIP stream (mc_create /
 *     mc_set_stream).  Calls that return results to host memory synchronize
 *     that stream; the device-output calls (mc_lookup_*, mc_sort_queue) do not.
 *   - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef MC_H
#define MC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum mc_status {
    MC_OK = 0,
    MC_EINVAL = -1,  /* invalid argument: non-increasing grid, density <= 0, bad id, size */
    MC_ENOMEM = -2,  /* device or host allocation failed */
    MC_EHIP = -3,    /* a HIP runtime call failed (text in mc_last_error) */
    MC_ELOST = -4,   /* more lost particles than mc_run_opts.max_lost */
    MC_ESTATE = -5,  /* call order: materials before geometry before runs */
    MC_ENODEV = -6,  /* no usable gfx950 device */
    MC_ERANGE = -7   /* a fixed-point mesh tally's range bound failed (see mc_run_batch) */
} mc_status;

typedef struct mc_ctx mc_ctx; /* opaque */

/* geometry, boundary, source and tally kinds */
enum { MC_GEOM_INFINITE = 0, MC_GEOM_LATTICE = 1, MC_GEOM_SLAB = 2 };
enum { MC_BC_REFLECT = 0, MC_BC_VACUUM = 1 };
enum { MC_SRC_POINT = 0, MC_SRC_BOX = 1, MC_SRC_BEAM = 2 };
enum { MC_TALLY_ENERGY = 0, MC_TALLY_PIN = 1, MC_TALLY_MESH = 2, MC_TALLY_SLAB = 3 };

/* tally ids for mc_get_tallies (MC_T_REACTION: with reaction channels,
 * n_mat * n_chan bins, material-major: the track-length rate sum of
 * w * d * Sigma_x over the flights in material m, channel x at m * n_chan + x) */
enum { MC_T_FLUX_TRACK = 0, MC_T_FLUX_COLLISION = 1, MC_T_GLOBAL = 2, MC_T_REACTION = 3 };

/* most reaction channels (mc_init_channels) */
#define MC_MAX_CHANNELS 16

/* bins of the MC_T_GLOBAL tally (each a per-source-particle mean) */
enum {
    MC_G_TRACK = 0,        /* sum of w*d over every flight (total track length) */
    MC_G_COLL_EST = 1,     /* sum of w/Sigma_t over collisions                  */
    MC_G_ABSORB = 2,       /* weight absorbed                                   */
    MC_G_CUTOFF = 3,       /* weight killed by the energy cutoff                */
    MC_G_LEAK = 4,         /* weight leaked through vacuum faces                */
    MC_G_TRACK_ABS = 5,    /* sum of w*d*Sigma_a                                */
    MC_G_NCOLL = 6,        /* collisions                                        */
    MC_G_NCROSS = 7,       /* surface crossings                                 */
    MC_G_LEAK_XHI = 8,     /* weight leaked through the x+ face                 */
    MC_G_LEAK_XHI_UNC = 9, /* the same, for particles that never collided       */
    MC_G_SPLIT = 10,       /* copies created by weight-window splitting         */
    MC_G_ROULETTE = 11,    /* particles killed by weight-window roulette        */
    MC_N_GLOBAL = 12
};

/* fate codes of mc_history.fate */
enum { MC_FATE_ABSORBED = 1, MC_FATE_CUTOFF = 2, MC_FATE_LEAKED = 3, MC_FATE_LOST = 4, MC_FATE_ROULETTE = 5 };

/*
 * Problem geometry, source and tally (one struct; unused members are ignored).
 *
 * MC_GEOM_INFINITE: one material everywhere, no surfaces.
 * MC_GEOM_LATTICE : nx*ny square cells of side `pitch` covering
 *   [0, nx*pitch] x [0, ny*pitch] x [z0, z1]; cell (i, j) holds a z-cylinder
 *   of radius `radius` (< pitch/2) about its centre filled with
 *   pin_material[j*nx + i] (-1: no cylinder), and moderator_material outside.
 *   A 2-level assembly lattice whose assembly pitch is a whole number of pin
 *   pitches is described as the equivalent flat lattice: each assembly's
 *   pin layout (its pin materials and its positions without a cylinder,
 *   such as water holes and guide tubes) fills pin_material at its cells.
 *   One pin radius and pitch hold for the whole lattice (no gaps between
 *   assemblies).
 * MC_GEOM_SLAB    : layers along x with edges x_edges[0..n_layers], infinite in
 *   y and z; layer l holds layer_material[l].
 * bc[6]           : boundary condition of the x-, x+, y-, y+, z-, z+ faces.
 * Source: MC_SRC_POINT (isotropic at source_pos), MC_SRC_BOX (uniform in
 *   source_box = {x0,x1,y0,y1,z0,z1}, isotropic), MC_SRC_BEAM (at source_pos
 *   along source_dir); every source particle starts at source_energy (eV),
 *   weight 1.
 * Tally (binning of MC_T_FLUX_TRACK and MC_T_FLUX_COLLISION):
 *   MC_TALLY_ENERGY: energy_edges[0..n_energy_bins] (eV, increasing; bins are
 *     [e_b, e_{b+1}), the top edge belongs to the last bin);
 *   MC_TALLY_PIN: one bin per lattice cell, scored inside its cylinder;
 *   MC_TALLY_MESH: mesh_dims[0]*mesh_dims[1]*mesh_dims[2] cells over mesh_box,
 *     x fastest; the track-length score of a flight is split over the cells
 *     it crosses;
 *   MC_TALLY_SLAB: one bin per layer.
 * energy_cutoff: particles whose energy falls below it are killed (eV).
 * All arrays are host memory, copied during mc_init_geometry.
 */
typedef struct mc_geometry_desc {
    int32_t kind;
    int32_t material;            /* MC_GEOM_INFINITE */
    int32_t nx, ny;              /* MC_GEOM_LATTICE  */
    double pitch, radius, z0, z1;
    const int32_t *pin_material;
    int32_t moderator_material;
    int32_t bc[6];
    int32_t n_layers;            /* MC_GEOM_SLAB     */
    const double *x_edges;
    const int32_t *layer_material;
    int32_t source_kind;
    double source_pos[3];
    double source_box[6];
    double source_dir[3];
    double source_energy;
    int32_t tally_kind;
    int32_t n_energy_bins;
    const double *energy_edges;
    int32_t mesh_dims[3];
    double mesh_box[6];
    double energy_cutoff;
} mc_geometry_desc;

/* Options of one mc_run_batch call (all-zero = defaults). */
typedef struct mc_run_opts {
    uint64_t in_flight;    /* particle-bank capacity; 0: min(n, 4,194,304), with weight
                              windows min(max(4 n, 4096), 1,048,576) (copies take free
                              slots).  The paper caps particles in flight and refills
                              from the batch (section 2, "In-Flight Particles"); its
                              GPUs peaked near 1e6, an MI355X keeps gaining to ~4e6
                              on lookup-bound problems (denser sorted queues). */
    uint64_t sort_min;     /* sort the lookup queue by (material, energy bin) when it holds
                              at least this many particles; 0: 262,144; UINT64_MAX or
                              2^30: never (tables that fit the caches gain less from the
                              sort than it costs) */
    int32_t no_tally;      /* 1: inactive batch (no flux tallies scored); global tallies
                              are still scored */
    int32_t time_kernels;  /* 1: time every lookup launch with HIP events (mc_get_stats) */
    int64_t max_events;    /* per-history event cap; past it the particle is killed as
                              lost; 0: 100,000 */
    uint64_t max_lost;     /* lost particles tolerated before MC_ELOST; 0: none tolerated */
    void *history_log;     /* device, nullable: n mc_history records, one per pid
                              (record k = pid first_pid + k) */
} mc_run_opts;

/* Per-history record written when mc_run_opts.history_log is set. */
typedef struct mc_history {
    int32_t fate, n_coll, n_cross, pad;
    uint64_t n_draws;      /* random numbers consumed */
    double E_final;        /* energy at death (eV) */
    double track;          /* total path length (cm) */
    double weight;         /* weight at death */
} mc_history;

/* Counters of the last mc_run_batch. */
typedef struct mc_stats {
    uint64_t iterations;        /* event-loop iterations */
    uint64_t lookups;           /* macroscopic lookups (particles looked up) */
    uint64_t nuclide_lookups;   /* sum over lookups of the material's nuclide count */
    uint64_t lookup_launches;   /* lookup-kernel launches */
    uint64_t sorted_lookups;    /* lookups done on a sorted queue */
    uint64_t lost;              /* particles killed by the event cap */
    uint64_t lookup_bytes;      /* algorithmic bytes of the lookups: per lookup
                                   36 + 56 * n_nuclides */
    double lookup_ms;           /* summed lookup-kernel time (time_kernels = 1), ms */
    double batch_ms;            /* wall time of the batch on the stream, ms */
    uint64_t tail_particles;    /* particles finished by the one-launch tail (their
                                   later lookups are not in the counters above; the
                                   tail runs analog batches without an importance
                                   grid only) */
    uint64_t mesh_underflow;    /* mesh-tally contributions (track length and
                                   collision estimator) that were positive but
                                   below the fixed-point resolution 2^-33 weight*cm
                                   and so added nothing */
    uint64_t flights;           /* particles the flight kernel advanced (one per
                                   alive particle and iteration; the tail's are
                                   not counted) */
    double advance_ms;          /* summed flight-kernel time (time_kernels = 1), ms */
    double cross_ms;            /* summed queue-split and surface-crossing time, ms */
    double collide_ms;          /* summed collision time (with its queue sort), ms */
} mc_stats;

/* Batch statistics of one tally (mc_get_tallies).  s1 and s2 are set by the
 * caller: when non-null they must hold n_bins doubles (host) and receive the
 * raw batch sums S1 = sum_b T_b and S2 = sum_b T_b^2 of the per-source-particle
 * batch values T_b -- with n_batches and histories, the state that
 * mc_set_tallies restores (checkpoint and resume between batches). */
typedef struct mc_tally_meta {
    uint64_t n_batches;
    uint64_t n_bins;
    uint64_t histories;    /* histories summed over all batches */
    double *s1, *s2;       /* caller-owned host arrays (nullable), filled by the call */
} mc_tally_meta;

/*
 * Device memory of a context: when given to mc_create, every device buffer
 * the library needs (tables, particle bank, queues, tallies, scratch) comes
 * from alloc and goes back through release; without it the library calls
 * hipMalloc / hipFree.  alloc(user, bytes, device, stream) returns device
 * memory of `device` usable on `stream` (the context's, or one of its event
 * loops' streams) or NULL (the call then fails with MC_ENOMEM); release(user,
 * ptr, device, stream) is called for each such pointer once no work that uses
 * it remains (the library synchronizes first).  Both may be called from the
 * library's event-loop threads.  The PyTorch binding passes its caching
 * allocator here.
 */
typedef struct mc_alloc {
    void *(*alloc)(void *user, size_t bytes, int device, void *stream);
    void (*release)(void *user, void *ptr, int device, void *stream);
    void *user;
} mc_alloc;

/*
 * Create a context on HIP device `device` (must be gfx950) that enqueues its
 * work on `hip_stream` (a hipStream_t; NULL = the device's null stream).
 * alloc (nullable, copied) supplies the context's device memory (see
 * mc_alloc).  *out receives the context; on failure *out is NULL and the
 * return value says why (MC_ENODEV, MC_EHIP, MC_ENOMEM).
 */
int mc_create(mc_ctx **out, int device, void *hip_stream, const mc_alloc *alloc);

/* Free every device buffer of the context (synchronizes its stream). */
void mc_destroy(mc_ctx *ctx);

/* Text of the last error on this context ("" if none); owned by the context. */
const char *mc_last_error(const mc_ctx *ctx);

/* Make later calls enqueue on `hip_stream`. */
int mc_set_stream(mc_ctx *ctx, void *hip_stream);

/*
 * Nuclide and material data (paper section 4.1: hundreds of nuclides per
 * material, whose per-nuclide lookups and sum form the dominant cost).
 *   n_nuc            number of nuclides (>= 1)
 *   grid_len[k]      points of nuclide k's energy grid (>= 2)
 *   E[k]             host, grid_len[k] fp64 energies (eV), strictly increasing
 *   sig_c[k], sig_s[k] host, grid_len[k] fp64 capture / elastic cross sections
 *                    (barns, >= 0) tabulated on E[k]; between points the
 *                    library interpolates linearly
 *   awr[k]           target mass ratio A (> 0)
 *   n_mat            number of materials (>= 1)
 *   mat_len[m]       nuclides in material m (>= 1)
 *   mat_nuc          concatenated nuclide ids of all materials, in material order
 *   mat_dens         concatenated atom densities (atoms/(barn cm), > 0)
 *   n_hash_bins      M, bins of the logarithmic hash grid over
 *                    [min_k E[k][0], max_k E[k][last]] (>= 1; 8192 typical)
 * Builds the per-material hash bounds on the host.  Replaces earlier data.
 * Errors: MC_EINVAL with the offending nuclide/material named.
 */
int mc_init_materials(mc_ctx *ctx, int32_t n_nuc, const int32_t *grid_len,
                      const double *const *E, const double *const *sig_c,
                      const double *const *sig_s, const double *awr, int32_t n_mat,
                      const int32_t *mat_len, const int32_t *mat_nuc, const double *mat_dens,
                      int32_t n_hash_bins);

/* Geometry, source and tally (see mc_geometry_desc): the constructive solid
 * geometry the particles are ray-traced through, surface by surface (paper
 * section 3: surface tracking; the lattice of pins of section 4.1), where
 * the source particles start, and what is tallied.  Requires materials.
 * Resets the tallies.  Errors: MC_EINVAL, MC_ESTATE. */
int mc_init_geometry(mc_ctx *ctx, const mc_geometry_desc *desc);

/*
 * Track histories with particle ids [first_pid, first_pid + n) to death and
 * add them to the tallies as one batch.  The histories run event by event
 * over the whole bank of particles in flight (paper section 2, "Event-Based
 * Parallelism": lookup, flight, crossing and collision kernels chosen from
 * event queues), the lookup queue sorted by material and energy (section 2,
 * "Sorting"), dead slots refilled from the batch until every history has
 * started (section 2, "In-Flight Particles").  Particle pid draws its random
 * numbers from the Philox4x32-10 stream keyed by `seed` with counter
 * (draw/2, lineage, pid), so a history does not depend on what else runs.
 * opts may be NULL (defaults).  Synchronizes the stream at the end.
 * Mesh tallies accumulate each batch in fixed point (2^-32 weight*cm); a batch
 * whose total weighted track length reaches 2^31 could wrap a bin, and then
 * the call returns MC_ERANGE (its values are already in the sums: reset or
 * restore the tallies, and run smaller batches).
 * Errors: MC_ESTATE (no geometry), MC_EINVAL, MC_ENOMEM, MC_EHIP, MC_ELOST,
 * MC_ERANGE.
 */
int mc_run_batch(mc_ctx *ctx, uint64_t seed, uint64_t first_pid, uint64_t n,
                 const mc_run_opts *opts);

/*
 * n_batches batches of n histories each, batch b holding pids [first_pid +
 * b n, first_pid + (b + 1) n): the same tallies, bit for bit, as n_batches
 * calls of mc_run_batch (each batch's value is formed from its own rows and
 * the statistics take the values in batch order).  With the tuning field
 * loops = L > 1 (analog transport) up to L batches run at once, each whole
 * batch on its own event loop (stream, host thread and bank), the next batch
 * to the first loop free -- the overlap the paper gets from several ranks per
 * GPU (section 2, "GPU Streams"): one batch's sparse tail runs beside another
 * batch's full queues.  mc_get_stats then describes the whole call (batch_ms:
 * its wall time; the counters summed).  history_log (opts) holds n_batches * n
 * records.  At most 2^20 batches per call.  Errors as mc_run_batch.
 */
int mc_run_batches(mc_ctx *ctx, uint64_t seed, uint64_t first_pid, uint64_t n, uint64_t n_batches,
                 const mc_run_opts *opts);

/*
 * Batch statistics of tally `tally_id` (MC_T_*) over every batch since the
 * last reset (paper section 2, "Tallying": tallies are scored in active
 * batches): mean[b] = S1/B and stderr_[b] = sqrt((S2/B - mean^2)/(B - 1)) of
 * the per-source-particle batch values (stderr_ is 0 when B < 2).
 * mean and stderr_ are host arrays of n_bins entries (n_bins must equal the
 * tally's bin count: MC_N_GLOBAL for MC_T_GLOBAL); either may be NULL; meta
 * may be NULL (and receives the raw sums when meta->s1 / meta->s2 are set).
 */
int mc_get_tallies(mc_ctx *ctx, int32_t tally_id, double *mean, double *stderr_, size_t n_bins,
                   mc_tally_meta *meta);

/*
 * Restore tally `tally_id` to raw batch sums read by mc_get_tallies (s1, s2:
 * host, n_bins doubles each, n_bins the tally's bin count) and set the
 * context's batch count and history total to n_batches and histories (shared
 * by all tallies: restore every tally with the same values).  Later batches
 * then add to the restored sums exactly as they would have added to the
 * originals, so a run stopped between batches and resumed in a new context
 * gives the same tallies bit for bit.  Errors: MC_ESTATE (no geometry; no
 * reaction channels for MC_T_REACTION), MC_EINVAL (id, n_bins, NULL arrays,
 * non-finite values, histories < n_batches).
 */
int mc_set_tallies(mc_ctx *ctx, int32_t tally_id, const double *s1, const double *s2, size_t n_bins,
                   uint64_t n_batches, uint64_t histories);

/* Zero every tally's batch sums. */
int mc_reset_tallies(mc_ctx *ctx);

/* Counters of the last mc_run_batch, or of the stand-alone lookups since
 * mc_set_timing (host struct). */
int mc_get_stats(mc_ctx *ctx, mc_stats *out);

/*
 * on = 1: zero the counters of mc_get_stats and, from then on, time every
 * lookup kernel that mc_lookup_macro launches with HIP events on the context's
 * stream and add it to those counters (lookups, nuclide_lookups,
 * lookup_launches, lookup_bytes, lookup_ms; each timed call synchronizes the
 * stream).  on = 0: stop timing the stand-alone calls.
 */
int mc_set_timing(mc_ctx *ctx, int32_t on);

/*
 * Reaction channels: n_chan further cross sections per grid point of every
 * nuclide (the per-nuclide reaction data a depletion calculation tallies,
 * paper section 2 "Tallying"; each adds to what every lookup gathers).  Each
 * channel is interpolated with the same grid index and fraction as the
 * capture and scattering cross sections and summed over the material's
 * nuclides in material order, times the densities; with channels every
 * lookup of mc_run_batch assembles them in the same pass, and the flights
 * score the MC_T_REACTION tally (track-length rates w * d * Sigma_x, per
 * material and channel) in active batches.  The problem-set path does not
 * use them.
 *   n_chan   0 .. MC_MAX_CHANNELS; 0 removes the channels (sig_x unused)
 *   sig_x    host, n_nuc pointers; sig_x[k] holds grid_len[k] * n_chan fp64
 *            values of nuclide k, point-major (channel x of point j at
 *            j * n_chan + x), finite and >= 0; copied during the call
 * mc_init_materials removes the channels.  Errors: MC_ESTATE (no materials),
 * MC_EINVAL (n_chan out of range, missing array, negative or non-finite
 * value), MC_ENOMEM.
 */
int mc_init_channels(mc_ctx *ctx, int32_t n_chan, const double *const *sig_x);

/*
 * Windowed-multipole cross sections with Doppler broadening computed on the
 * fly (the compute-bound alternative to tabulated data that the paper points
 * to in section 4.1).  In u = sqrt(E) (eV^1/2) a nuclide's microscopic
 * capture / scattering cross section at temperature T is
 *   sigma_x(E, T) = (1/E) sum_j Re[ r_x,j sqrt(pi) beta w(beta (u - p_j)) ]
 *                   + sum_n b_x,w,n u^(n-1),     beta = sqrt(A / (k_B T)),
 * w the Faddeeva function (evaluated by Weideman's rational series, 32 terms),
 * the sum over the poles of the window w holding u (windows split [u_lo,
 * u_hi] evenly; u outside clamps to the first / last window).  As T -> 0 each
 * pole term tends to Re[r i / (u - p)] / E.  These data stand apart from the
 * tabulated materials (their own nuclides and materials).
 */
typedef struct mc_mp_nuclide {
    int32_t n_poles;      /* >= 0 */
    int32_t n_windows;    /* >= 1 */
    int32_t n_bg;         /* background coefficients per window, 0 .. 8 */
    int32_t reserved;
    double u_lo, u_hi;    /* window range in sqrt(eV), 0 < u_lo < u_hi */
    const double *poles;  /* host, [n_poles][2] (re, im), Im < 0 */
    const double *res_c;  /* host, [n_poles][2] capture residues (barn eV) */
    const double *res_s;  /* host, [n_poles][2] scattering residues */
    const int32_t *win;   /* host, [n_windows][2] pole ranges [start, end) */
    const double *bg_c;   /* host, [n_windows][n_bg] coefficients of u^-1, u^0, ... */
    const double *bg_s;
} mc_mp_nuclide;

/*
 * Load multipole nuclides (copied during the call) and materials of them:
 * mat_len / mat_nuc / mat_dens as in mc_init_materials, mat_temp[m] the
 * temperature of material m in kelvin (> 0).  Replaces earlier multipole
 * data.  Errors: MC_EINVAL (counts, ranges, Im p >= 0, non-finite data, ids,
 * densities, temperatures), MC_ENOMEM.
 */
int mc_init_multipole(mc_ctx *ctx, int32_t n_nuc, const mc_mp_nuclide *nucs, const double *awr, int32_t n_mat,
                      const int32_t *mat_len, const int32_t *mat_nuc, const double *mat_dens,
                      const double *mat_temp);

/*
 * Macroscopic multipole cross sections of n (energy, material) pairs: sig_a /
 * sig_s (device, n fp64) = sum over the material's nuclides, in material
 * order, of density * sigma_c / sigma_s at the material's temperature.
 * E, mat device inputs (n each).  poles_evaluated (nullable, host): the
 * number of pole terms summed (synchronizes the stream).  Timed like
 * mc_lookup_macro when mc_set_timing is on (lookups, launches, ms).  Errors:
 * MC_ESTATE (no multipole data), MC_EINVAL.
 */
int mc_lookup_multipole(mc_ctx *ctx, size_t n, const double *E, const int32_t *mat, double *sig_a, double *sig_s,
                        uint64_t *poles_evaluated);

/*
 * Unionized-grid lookups (the alternative to per-nuclide searches the paper
 * names among the lookup accelerations, section 3): per material, the sorted
 * union U of its nuclides' energy grids with its own hash bounds, and per
 * union point u a row of every nuclide's interval at U_u (4 B per union point
 * and nuclide).  A lookup then searches the union grid once and reads each
 * nuclide's interval from the row instead of searching it: the same
 * intervals, interpolation and sums, so the same results bit for bit.
 *   on      1: build the tables (host work, then device memory) and use them
 *           for every macroscopic lookup of the context (transport and
 *           mc_lookup_macro; the per-nuclide outputs of mc_lookup_nuclides,
 *           the reaction channels and the collision's re-gathers keep the
 *           hash search); 0: free them.
 *   bytes   (nullable) device bytes of the tables
 * mc_init_materials removes them.  Errors: MC_ESTATE (no materials), MC_EINVAL
 * (a material's union grid above 2^32 points or 2^34 row entries),
 * MC_ENOMEM.
 */
int mc_set_union_grid(mc_ctx *ctx, int32_t on, uint64_t *bytes);

/*
 * The channel lookup on its own: for n (energy, material) pairs, out[i *
 * n_chan + x] = sum over the material's nuclides of density * channel x
 * (device, n * n_chan fp64), and, when non-null, sig_a / sig_s as in
 * mc_lookup_macro (device, n fp64 each).  Timed like mc_lookup_macro (with
 * 8 B per channel and lookup and 16 B per channel and nuclide added to the
 * algorithmic bytes).  Errors: MC_ESTATE (no materials or no channels),
 * MC_EINVAL.
 */
int mc_lookup_channels(mc_ctx *ctx, size_t n, const double *E, const int32_t *mat, double *out, double *sig_a,
                       double *sig_s);

/*
 * Macroscopic cross sections of n (energy, material) pairs, the lookup step on
 * its own (paper section 2, "Sorting": the lookup is typically the most
 * expensive part of the simulation).
 *   E         device, n fp64 energies (eV)
 *   mat       device, n int32 material ids
 *   sig_a     device, n fp64 outputs: sum over the material's nuclides of
 *             density * capture cross section, in material order
 *   sig_s     device, n fp64 outputs: the same for elastic scattering
 *   sorted    1: sort the pairs by (material, hash bin) on the device first
 *             (needs no caller memory); 0: process them in the given order
 * Errors: MC_ESTATE (no materials), MC_EINVAL (bad material id on the host
 * side is not checked: ids must be in [0, n_mat)).
 */
int mc_lookup_macro(mc_ctx *ctx, size_t n, const double *E, const int32_t *mat, double *sig_a,
                    double *sig_s, int32_t sorted);

/*
 * mc_lookup_macro without any allocation, for callers that cannot allocate
 * device memory during the call (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same arguments, kernels and
 * results as mc_lookup_macro; the sort's scratch (keys, permutation, radix
 * partials) lives in a static device array of the library, one per GPU,
 * allocated when the library's code is loaded and held until the process
 * ends (MC_NOALLOC_SCRATCH_BYTES).  The call allocates nothing (no hipMalloc,
 * no caller allocator, no events) and does not honour mc_set_timing.
 *   n        at most MC_NOALLOC_MAX_LOOKUPS; larger n is rejected
 * Every call on a GPU shares that GPU's array: calls that overlap on one GPU
 * (from several contexts, streams or threads) race and give wrong results;
 * serialize them.  The array's device address is looked up once per GPU by
 * mc_create (which fails with MC_EHIP if it cannot be had).  Errors:
 * MC_ESTATE (no materials), MC_EINVAL (n above the maximum, null E or mat),
 * MC_EHIP.
 */
#define MC_NOALLOC_MAX_LOOKUPS (1u << 20)
#define MC_NOALLOC_SCRATCH_BYTES (30u << 20)
int mc_lookup_macro_noalloc(mc_ctx *ctx, size_t n, const double *E, const int32_t *mat, double *sig_a,
                            double *sig_s, int32_t sorted);

/*
 * Per-nuclide results of the same lookup for n pairs that all use material
 * `mat` (n_k = its nuclide count):
 *   E        device, n fp64 energies
 *   idx      device, n*n_k int32: grid index i(E) = max{j : E_j <= E} clamped
 *            to [0, N-2], for nuclide q of the material at [p*n_k + q]
 *   sig_c, sig_s device, n*n_k fp64 interpolated microscopic cross sections
 * Any output pointer may be NULL.
 */
int mc_lookup_nuclides(mc_ctx *ctx, int32_t mat, size_t n, const double *E, int32_t *idx,
                       double *sig_c, double *sig_s);

/*
 * The sort step on its own (paper section 2, "Sorting"): key[p] = mat[p] * M +
 * b(E[p]) with b the hash bin, then perm receives 0..n-1 ordered by key
 * (stable: equal keys keep their input order) and keys_sorted the keys in that
 * order.
 *   E, mat      device inputs (n each)
 *   perm        device, n uint32 outputs
 *   keys_sorted device, n uint32 outputs (nullable)
 */
int mc_sort_queue(mc_ctx *ctx, size_t n, const double *E, const int32_t *mat, uint32_t *perm,
                  uint32_t *keys_sorted);

/*
 * Host-only helper (no device needed): the hash bounds the library builds for
 * one grid.  lo[b] = i(E_b) for b = 0..M-1, E_b = emin * exp(b * ln(emax/emin)/M),
 * and lo[M] = N-2, where i() is the grid index of mc_lookup_nuclides.  lo is a
 * host array of M + 1 entries.
 */
int mc_hash_bounds(const double *E, int32_t N, double emin, double emax, int32_t M, int32_t *lo);

/*
 * Launch-shape parameters of the kernels (the autotuner's search space).
 * Zero fields keep the library default.  They change speed only: histories
 * are the same for every setting, and tallies agree to summation order.
 *   lookup_ilp     nuclides each lane looks up in lockstep in the lookup
 *                  kernel (1, 2 or 4; default 2)
 *   tail_particles when no history remains to start and at most this many
 *                  particles are in flight, the remaining histories are
 *                  finished by one kernel launch in which each lane runs its
 *                  particle to the end (0: default 131,072; -1: never)
 *   sort_min       default of mc_run_opts.sort_min (0: 262,144; 2^30: never)
 *   in_flight      default of mc_run_opts.in_flight (0: 4,194,304; 1,048,576
 *                  with weight windows)
 *   set_tile_histories  histories per work item of the problem-set kernel,
 *                  a multiple of 256 (0: 256)
 *   set_grid       persistent workgroups of the problem-set kernel (0: two
 *                  per compute unit)
 *   collide_sort_min  sort the collide queue (by material and energy bin, for
 *                  the collision's re-gathers) when at least this many
 *                  particles are alive (0: the lookup queue's sort_min;
 *                  2^30: never)
 *   loops          event loops run at once in mc_run_batch (0 or 1: one;
 *                  at most 8): loop l takes the l-th contiguous share of the
 *                  batch's pids on its own stream and host thread, with its
 *                  own bank of in_flight slots, sharing the tables; the
 *                  batch tallies sum the loops' rows in loop order, so the
 *                  histories are the same for any count and the tallies
 *                  differ only by summation order (reruns with the same count
 *                  are bitwise identical).  The paper runs several ranks per
 *                  GPU for the same overlap (section 2, "GPU Streams").
 *                  Analog batches only (one loop with weight windows or an
 *                  importance grid), and at least 4096 histories per loop.
 */
typedef struct mc_tuning {
    int32_t lookup_ilp;
    int32_t tail_particles;
    int32_t sort_min;
    int32_t in_flight;
    int32_t set_tile_histories;
    int32_t set_grid;
    int32_t collide_sort_min;
    int32_t loops;
} mc_tuning;

/* Set (mc_set_tuning) or read (mc_get_tuning) the context's launch shapes.
 * Errors: MC_EINVAL for a value outside the ranges above. */
int mc_set_tuning(mc_ctx *ctx, const mc_tuning *t);
int mc_get_tuning(mc_ctx *ctx, mc_tuning *t);

/*
 * Autotuner of the single-problem path: times batches of n histories (pids
 * from first_pid, key seed) per candidate, per batch: 12 through
 * mc_run_batches, or for n >= 2^22 two single batches through mc_run_batch
 * (how such batches run: one at a time, split over the loops), searching one
 * parameter at a time (two sweeps, in this order) over loops {1, 2, 3, 4},
 * tail_particles {8192, 32768, 131072, 262144}, sort_min {4096, 16384,
 * 65536, 262144, never}, lookup_ilp {1, 2, 4}, in_flight {n/4, n/3, n/2,
 * 2^20, 2^22, n} (each at most n and 2^24; the search starts from
 * min(n, 2^22)) and collide_sort_min {0, never}, keeps the fastest in the
 * context (mc_set_tuning) and returns it in *best.  The tallies are reset afterwards.  cache_path (nullable) names a
 * text file of one line per tuned problem: when it holds the signature of
 * this problem and device, the stored setting is used without timing; else
 * the result is appended.  Requires materials and geometry.
 */
int mc_autotune(mc_ctx *ctx, uint64_t seed, uint64_t first_pid, uint64_t n, const char *cache_path,
                mc_tuning *best);

/*
 * Problem set: many small independent fixed-source problems run together in
 * one persistent kernel (workgroups pull (problem, history range) tiles from a
 * queue until none is left), the batching layer that stands in for the
 * paper's concurrent streams on one GPU (section 2, "GPU Streams") and its
 * refill of in-flight particles (section 2, "In-Flight Particles").
 * Each problem has its own nuclides, materials (ids local to the problem),
 * geometry, source, tally (not a mesh), histories per batch and seed; batch b
 * of problem p runs pids first_pid + b * histories + [0, histories).  A
 * problem's histories are the ones mc_run_batch would run for it alone.
 */
typedef struct mc_problem_desc {
    int32_t n_nuc;
    const int32_t *grid_len;
    const double *const *E;
    const double *const *sig_c;
    const double *const *sig_s;
    const double *awr;
    int32_t n_mat;
    const int32_t *mat_len;
    const int32_t *mat_nuc;
    const double *mat_dens;
    const mc_geometry_desc *geometry;
    uint64_t histories;
    uint64_t seed;
    uint64_t first_pid;
} mc_problem_desc;

/* Upload a problem set (host arrays, copied); replaces an earlier set and
 * zeroes its tallies.  Errors: MC_EINVAL naming the problem. */
int mc_set_problem_set(mc_ctx *ctx, int32_t n_problems, const mc_problem_desc *problems,
                       int32_t n_hash_bins);

typedef struct mc_set_opts {
    int32_t use_graph;     /* 1: replay a captured hipGraph of the whole batch (zeroing,
                              persistent kernel, statistics), captured on first use */
    int32_t pad;
    int64_t max_events;    /* per-history event cap (0: 100,000) */
    void *history_log;     /* device, nullable: one mc_history per history of the
                              batch, problem after problem in input order (not with
                              use_graph) */
} mc_set_opts;

/* Run one batch of every problem of the set.  Synchronizes the stream. */
int mc_run_problem_set(mc_ctx *ctx, const mc_set_opts *opts);

/* Batch statistics of one problem's tally (as mc_get_tallies). */
int mc_get_problem_tallies(mc_ctx *ctx, int32_t problem, int32_t tally_id, double *mean,
                           double *stderr_, size_t n_bins, mc_tally_meta *meta);

/* Zero the set's tallies and restart its batch count at 0. */
int mc_reset_problem_set(mc_ctx *ctx);

/*
 * Autotuner of the problem set: times one batch per candidate over
 * set_tile_histories {256, 512, 1024, 2048} x set_grid {1, 2, 4, 8 per
 * compute unit}, keeps the fastest, resets the set (mc_reset_problem_set).
 * cache_path as for mc_autotune.
 */
int mc_autotune_problem_set(mc_ctx *ctx, const char *cache_path, mc_tuning *best);

/*
 * Importance network (learned importance map for weight windows).
 *
 * A 4 -> 64 -> 64 -> 1 perceptron with SiLU hidden activations predicting
 * ln I from the features (x/L, clip(y/L, -1, 1), clip(z/L, -1, 1),
 * (ln E - ln 1e-5) / ln(2e12)).  Parameters are one flat FP32 array of
 * MC_MLP_NPAR values in the order W1[4][64], b1[64], W2[64][64], b2[64],
 * w3[64], b3 (W[k][j]: input k -> output j).  The kernels keep BF16 copies
 * of W1, W2 and w3, feed the 64x64 products to the matrix cores with FP32
 * accumulation, and round the inputs and the first hidden activation to
 * BF16; biases and everything else are FP32.
 */
enum { MC_MLP_NPAR = 4545 };

/* Load the parameters (host array of MC_MLP_NPAR floats, copied) and reset
 * the Adam state.  Errors: MC_EINVAL (NULL or a non-finite value). */
int mc_mlp_set(mc_ctx *ctx, const float *params);

/* Copy the current FP32 parameters into a host array of MC_MLP_NPAR floats.
 * Errors: MC_ESTATE (no network loaded). */
int mc_mlp_get(mc_ctx *ctx, float *params);

/* ln I of n feature vectors: features is a device array [n][4] (FP32, row
 * major), out a device array [n].  Asynchronous on the context's stream; the
 * caller owns both buffers.  Errors: MC_ESTATE, MC_EINVAL (n >= 2^31). */
int mc_mlp_forward(mc_ctx *ctx, size_t n, const float *features, float *out);

/* Gradient of the weighted squared error sum_i w_i (y_i - t_i)^2 / sum_i w_i
 * over n samples (device arrays: features [n][4], target [n], weight [n]).
 * grad (host, MC_MLP_NPAR floats, flat order) and loss (host) may be NULL.
 * Summation order is fixed: results are reproducible run to run.
 * Errors: MC_ESTATE, MC_EINVAL (n == 0 or n >= 2^24). */
int mc_mlp_grad(mc_ctx *ctx, size_t n, const float *features, const float *target, const float *weight,
                float *grad, float *loss);

/* Full-batch training: `steps` Adam steps (beta1 0.9, beta2 0.999, eps 1e-8,
 * step counter continuing from earlier calls since mc_mlp_set) at learning
 * rate lr on the samples above.  loss_curve (host, `steps` floats, may be
 * NULL) receives the loss before each step.  Synchronous.
 * Errors: MC_ESTATE, MC_EINVAL. */
int mc_mlp_train(mc_ctx *ctx, size_t n, const float *features, const float *target, const float *weight,
                 int32_t steps, float lr, float *loss_curve);

/*
 * Weight windows and the forward importance estimate.
 *
 * The paper's transport is analog; weight windows are the textbook
 * split / roulette game driven by an importance map ln I(x, y, z, E).  The
 * window at a point is w_L = exp(ln I_src - ln I) / kappa, w_U = ratio * w_L,
 * w_S = (w_L + w_U) / 2, with ln I_src the map at the source point (the box
 * centre for a box source), evaluated at the start of every mc_run_batch.  It
 * is checked after every collision the particle survives and every crossing
 * it does not leak through: above w_U the particle splits into
 * n = min(n_max, ceil(w / w_U)) copies of weight w / n (none when the
 * history already holds `depth` pending splits); below w_L it plays roulette
 * with one draw and survives at w_S with probability w / w_S.  Pending copies
 * wait on a last-in first-out stack of the history and run when the copy
 * ahead of them ends; copy k of split number s of a copy of lineage a draws
 * from lineage child_lineage(a, s, k) of the same pid (MurmurHash3's 32-bit
 * finaliser of the three, never 0), so a history with all its copies depends
 * on (seed, pid) only.  Features: f_x = x / length, f_E = (ln E - ln 1e-5) /
 * ln(2e12); the network sees (x, clip(y), clip(z)) / length and f_E.
 *
 * Forward importance estimate (after Booth), on imp_nx x-bins over
 * [imp_x0, imp_x1) by imp_ne ln E-bins over [1e-5, 2e7] eV (points outside
 * fall in the end bins): the weight of a copy entering a cell for the first
 * time (copies inherit what their parent entered) adds to den[cell]; weight
 * leaking through the x+ face adds to num[cell] (and 1 to cnt[cell]) of every
 * cell that copy has entered.  num / den estimates the expected score of unit
 * weight entering the cell.  Cells are indexed e * imp_nx + x.  The sums use
 * FP64 atomics: they are exact up to the order of the additions.
 */
enum { MC_WW_OFF = 0, MC_WW_LINEAR = 1, MC_WW_MLP = 2 };

typedef struct {
    int32_t kind;          /* MC_WW_OFF, MC_WW_LINEAR (ln I = lin[0] + lin[1] f_x + lin[2] f_E)
                              or MC_WW_MLP (the context's network, mc_mlp_set)          */
    int32_t n_max;         /* most copies per split, 2..1000                              */
    int32_t depth;         /* most pending splits per history, 1..64                      */
    int32_t imp_nx;        /* importance grid x-bins, 0 (no estimate) .. 256              */
    int32_t imp_ne;        /* importance grid ln E-bins, 1..64 when imp_nx > 0           */
    int32_t reserved;
    double lin[3];
    double length;         /* feature scale (cm), > 0                                     */
    double kappa;          /* w_L at the source point is 1 / kappa, > 0                   */
    double ratio;          /* w_U / w_L, > 1                                               */
    double imp_x0, imp_x1; /* x range of the importance grid                              */
    double ln_lo, ln_hi;   /* ln I (either kind, the source point too) is clamped to
                              [ln_lo, ln_hi] when ln_lo < ln_hi: a fitted map is trusted
                              over the span of its targets only                           */
} mc_ww_desc;

/* Configure (or, with NULL or kind MC_WW_OFF and imp_nx 0, remove) the
 * windows and the estimate for the following mc_run_batch calls; zeroes the
 * importance sums.  The problem-set path (mc_run_problem_set) stays analog.
 * Device memory for the pending copies: depth x in-flight slots x ~100 B
 * (plus 2 B per ln E-bin with the estimate on).  Errors: MC_EINVAL naming the
 * field; MC_ESTATE from mc_run_batch when MC_WW_MLP is set and no network is
 * loaded. */
int mc_set_weight_windows(mc_ctx *ctx, const mc_ww_desc *desc);

/* The bootstrap importance map of a deep-penetration problem from an analog
 * pilot: with R0 the mean of the MC_T_GLOBAL bin MC_G_LEAK_XHI (weight
 * leaking through the x+ face per source particle) over the context's
 * batches and N their histories, *slope = -ln(max(R0, 1/N)): the linear map
 * ln I = slope * f_x makes the importance of the far face relative to the
 * source that of the pilot's response (or of one history in N when none
 * scored).  Errors: MC_ESTATE (no geometry or no batch). */
int mc_ww_bootstrap_slope(mc_ctx *ctx, double *slope);

/* Importance sums since the last mc_set_weight_windows / tally reset, into
 * host arrays of n_cells = imp_nx * imp_ne doubles (each may be NULL).
 * Errors: MC_ESTATE (no grid), MC_EINVAL (n_cells). */
int mc_get_importance(mc_ctx *ctx, double *num, double *den, double *cnt, size_t n_cells);

/*
 * Training the network on the forward importance estimate.
 *
 * Samples: every cell of the importance grid with at least min_credits
 * detector credits (cnt) gives `replicas` samples, cells in index order
 * (e * nx + x): features (x centre / length, f_y, f_z, (e + 1/2) / ne), target
 * ln(num / den), weight 1 / (1 / cnt + rel_floor^2) (the inverse relative
 * variance of the ratio, floored).  The slab is invariant in y and z, so f_y
 * and f_z are drawn uniform on [-1, 1]: draws 2r and 2r + 1 of the Philox
 * stream (key seed, pid = cell, lineage 0x5EED0002).
 */
typedef struct {
    int32_t steps;      /* Adam steps, >= 1                                   */
    int32_t replicas;   /* samples per cell, 1..64                            */
    float lr;           /* Adam learning rate, > 0                            */
    float pad;
    double min_credits; /* cells with fewer credits are left out, >= 1        */
    double rel_floor;   /* relative-error floor of the weights, >= 0          */
    double length;      /* feature scale (cm), the windows' length            */
    uint64_t seed;      /* Philox key of the (f_y, f_z) draws                 */
} mc_train_opts;

/* Initial network: W1 ~ U(-1/2, 1/2), W2 and w3 ~ U(-1/8, 1/8), biases 0
 * (parameter j is 2u - 1 scaled, u draw 0 of pid j, lineage 0x5EED0001 of
 * key seed); Adam state reset. */
int mc_mlp_init(mc_ctx *ctx, uint64_t seed);

/* Training samples from host importance sums num, den, cnt [ne][nx] (x-bins
 * over [x0, x1)) into caller-owned device arrays features [nx ne replicas][4],
 * target and weight [nx ne replicas]; *n_samples (host) receives the count.
 * Errors: MC_EINVAL. */
int mc_importance_samples(mc_ctx *ctx, const double *num, const double *den, const double *cnt, int32_t nx,
                          int32_t ne, double x0, double x1, const mc_train_opts *opts, float *features,
                          float *target, float *weight, int32_t *n_samples);

/* Build the samples from the context's importance sums (mc_set_weight_windows
 * grid, accumulated by mc_run_batch) on the device and train the context's
 * network on them (opts->steps full-batch Adam steps, as mc_mlp_train).
 * loss_curve (host, steps floats), n_samples and target_range (host, the
 * smallest and largest target: the span to clamp the windows' ln I to) may be
 * NULL.  Synchronous.  Errors: MC_ESTATE (no network, no grid, or no cell with
 * enough credits), MC_EINVAL. */
int mc_importance_train(mc_ctx *ctx, const mc_train_opts *opts, float *loss_curve, int32_t *n_samples,
                        float *target_range);

/* Library version string. */
const char *mc_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MC_H */
