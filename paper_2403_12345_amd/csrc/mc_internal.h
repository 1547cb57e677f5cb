// mc_internal.h -- launch wrappers shared by the C-ABI layer and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mc_device.h"
#include "mc_mlp.h"
#include "mc_ww.h"

namespace mc {

struct LookupLaunch {
    XsDev xs;
    const uint32_t *list = nullptr;
    const uint32_t *keys = nullptr;
    const uint32_t *n_ptr = nullptr;
    uint32_t n_bound = 0;
    const double *E = nullptr;
    const int32_t *mat = nullptr;
    double *Sa = nullptr, *Ss = nullptr;
    uint8_t *flags = nullptr;
    int32_t *idx_out = nullptr;
    double *sc_out = nullptr, *ss_out = nullptr;
    unsigned long long *nuc_count = nullptr;
    int32_t ilp = 4;  // nuclides looked up in lockstep per lane (1, 2 or 4)
    double *cp = nullptr;     // scattering-sum checkpoints [slot][CP_MAX] (transport lookups only)
    double *sx = nullptr;     // reaction channels [p][n_chan] (when the tables have channels)
};

hipError_t launch_fill_u8(uint8_t *p, size_t n, uint8_t v, hipStream_t st);
hipError_t launch_fill_u32(uint32_t *p, size_t n, uint32_t v, hipStream_t st);
hipError_t launch_fill_f64(double *p, size_t n, double v, hipStream_t st);
hipError_t launch_slots_count(const BankDev &b, hipStream_t st);
hipError_t launch_slots_queue(const BankDev &b, const GeomDev &g, const WwDev &W, Counters *ctr, int cur,
                              uint64_t first_pid, uint64_t n_hist, uint64_t seed, uint32_t new_bound,
                              hipStream_t st);
// Scratch of the radix sort of up to `cap` items.
struct SortBufs {
    uint32_t *kA = nullptr, *kB = nullptr, *vA = nullptr, *vB = nullptr;
    uint32_t *tile_hist = nullptr;    // [tiles][256]
    uint32_t *chunk_total = nullptr;  // [chunks][256], kept zero between sorts
    uint32_t *chunk_off = nullptr;    // [chunks + 1][256]: per-chunk offsets, then the digit bases
};
// Windowed-multipole macroscopic cross sections of n (energy, material) pairs.
hipError_t launch_lookup_mp(const MpDev &mp, uint32_t n, const double *E, const int32_t *mat, double *Sa,
                            double *Ss, unsigned long long *pole_count, hipStream_t st);
size_t sort_tile_count(size_t n);
size_t sort_chunk_count(size_t n);
// Stable sort of the n (<= n_bound) items list[i] (or i) by key = mat * M + hash bin of E;
// out_list receives the items, out_keys the keys (both required).
hipError_t launch_sort(const XsDev &xs, const uint32_t *list, const uint32_t *n_ptr, uint32_t n_bound,
                       const double *E, const int32_t *mat, const SortBufs &sb, uint32_t n_keys,
                       uint32_t *out_list, uint32_t *out_keys, hipStream_t st);
hipError_t launch_lookup(const LookupLaunch &l, hipStream_t st);
hipError_t launch_advance(const BankDev &b, const GeomDev &g, const TallyDev &t, const WwDev &W, const Counters *ctr,
                          uint32_t n_bound, uint64_t seed, int64_t max_events, int32_t log_on, bool cross,
                          HistLog *log, uint64_t first_pid, unsigned long long *lost, hipStream_t st);
hipError_t launch_split(const BankDev &b, Counters *ctr, uint32_t n_bound, hipStream_t st);
hipError_t launch_cross(const BankDev &b, const GeomDev &g, const TallyDev &t, const WwDev &W, const Counters *ctr,
                        uint32_t n_bound, uint64_t seed, HistLog *log, uint64_t first_pid, unsigned long long *lost,
                        hipStream_t st);
hipError_t launch_collide(const BankDev &b, const uint32_t *list, const XsDev &xs, const GeomDev &g,
                          const TallyDev &t, const WwDev &W, const Counters *ctr, uint32_t n_bound, uint64_t seed,
                          HistLog *log, uint64_t first_pid, hipStream_t st);
hipError_t launch_tail(const BankDev &b, const XsDev &xs, const GeomDev &g, const TallyDev &t, const Counters *ctr,
                       uint32_t n_bound, uint64_t seed, int64_t max_events, HistLog *log, uint64_t first_pid,
                       unsigned long long *lost, hipStream_t st);
// Weight windows: pending copies of every slot's stack into the copy bank.
hipError_t launch_ww_flush(const BankDev &b, const WwDev &W, Counters *ctr, hipStream_t st);
// ln I at the source point into *out (device), for the weight windows.
hipError_t launch_ww_source(const WwDev &W, const GeomDev &g, double *out, hipStream_t st);
// Many independent problems (batching layer).
struct SetProblem {
    GeomDev g;          // material ids index the shared tables
    uint64_t seed;      // Philox key of the problem
    uint64_t histories; // per batch
    uint64_t pid_base;  // batch b runs pids pid_base + b * histories + [0, histories)
    uint64_t log_off;   // first record of the problem in the history log
    uint32_t first_tile, n_tiles;
    uint64_t stat_off;  // first of the problem's 2 n_bins + N_GLOBAL batch sums
};
struct SetTile {
    int32_t problem;
    uint32_t first, count;  // histories [first, first + count) of the problem's batch
    uint64_t row;           // offset (doubles) of the tile's tl / coll rows
};
struct SetDev {
    const SetProblem *problems;
    const SetTile *tiles;
    int32_t n_problems;
    uint32_t n_tiles;
    double *tl, *coll, *glob;     // tile rows
    size_t n_rows_doubles;        // doubles in tl (and coll)
    double *S1, *S2;              // per-problem batch sums
    uint32_t *next_tile;          // work-queue counter
    uint64_t *batch;              // batches run so far
    HistLog *log;                 // nullable
    unsigned long long *lost;
};
hipError_t launch_problem_set(const SetDev &set, const XsDev &xs, int64_t max_events, uint32_t grid,
                              int32_t max_bins, hipStream_t st);
// importance network
hipError_t launch_mlp_forward(const MlpDev &m, uint32_t n, const float *X, float *Y, hipStream_t st);
size_t mlp_partial_floats(uint32_t n);
hipError_t launch_mlp_wsum(const float *W, uint32_t n, float *inv_wsum, hipStream_t st);
hipError_t launch_mlp_grad(const MlpDev &m, uint32_t n, const float *X, const float *T, const float *W,
                           const float *inv_wsum, float *partial, float *grad_and_loss, hipStream_t st);
hipError_t launch_mlp_adam(float *theta, float *mom, float *vel, const float *grad, int step, float lr, uint16_t *W1,
                           uint16_t *W2, uint16_t *W2t, uint16_t *w3, hipStream_t st);
hipError_t launch_mlp_sync(const float *theta, uint16_t *W1, uint16_t *W2, uint16_t *W2t, uint16_t *w3, hipStream_t st);
constexpr uint32_t MLP_INIT_LINEAGE = 0x5EED0001u;    // Philox lineage of the initial parameters
constexpr uint32_t IMP_SAMPLE_LINEAGE = 0x5EED0002u;  // Philox lineage of the (y, z) replicas
hipError_t launch_mlp_init(float *theta, uint64_t seed, hipStream_t st);
struct ImpSampleArgs {
    const double *num, *den, *cnt;  // [ne][nx] importance sums
    int32_t nx, ne;
    double x0, x1, length;
    int32_t replicas;
    double min_credits, rel_floor;
    uint64_t seed;
    float *X, *T, *W;                // [cells * replicas][4], [..], [..]
    int32_t *n_out;                  // samples written
    float *range_out;                // [2] smallest and largest target
};
hipError_t launch_imp_samples(const ImpSampleArgs &a, hipStream_t st);
// S1 += T_b, S2 += T_b^2 over the batch values T[b * stride + off + k], b in order.
hipError_t launch_batch_accum_strided(const double *T, int32_t n_b, int32_t stride, int32_t off, int32_t n_cols,
                                      double *S1, double *S2, hipStream_t st);
hipError_t launch_batch_stats(const double *rows, int32_t n_rows, int32_t n_cols, const double *direct,
                              double *partial, double inv_n, double *S1, double *S2, hipStream_t st);

}  // namespace mc
