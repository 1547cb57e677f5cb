// mc_ww.h -- weight windows and the forward importance estimate on the GPU.
//
// Weight windows (the textbook split / roulette game; the paper's transport
// is analog and says nothing of it): the window at a point follows from an
// importance map ln I(x, y, z, E), w_L = exp(ln I_src - ln I) / kappa,
// w_U = ratio * w_L, w_S = (w_L + w_U) / 2.  A copy heavier than w_U is split
// into n = min(n_max, ceil(w / w_U)) copies of weight w / n (unless `depth`
// splits already lie on its line from the source particle); one goes on, the
// other n - 1 are pushed on the slot's stack of pending splits.  A copy
// lighter than w_L plays roulette (one draw) and survives at w_S with
// probability w / w_S.  Checks happen after a collision the particle survives
// and after a crossing it does not leak through.  Copy k of split number s of
// a copy of lineage a draws from the stream of lineage child_lineage(a, s, k)
// of the same pid, so every copy is fixed by (seed, pid) and its line alone,
// whatever slot runs it and when.
//
// Pending copies run in parallel: after every event step the stacks are
// flushed, in slot order, into a copy bank, and the refill step gives free
// slots copies from the bank before new source particles.  When the bank is
// full the stacks keep their records and a slot runs its own pending copies
// (last in, first out) when its copy ends.
//
// Forward importance estimate (after Booth): on a grid of x-bins by ln E-bins
// each copy remembers which cells it (or the copy it was split from) has
// entered; the weight that first enters a cell adds to that cell's
// denominator, a score (weight leaking through the x+ face) adds to the
// numerator of every cell entered.  I(cell) = numerator / denominator is the
// expected score of unit weight entering the cell.  Energies only decrease
// (elastic scattering off targets at rest) and paths are continuous, so the
// cells a copy has entered at one E-bin form one interval of x-bins: a copy
// keeps one (lo, hi) byte pair per E-bin instead of a bit per cell.
#pragma once

#include "mc_device.h"
#include "mc_mlp.h"
#include "mc_physics.h"

#pragma clang fp contract(off)

namespace mc {

enum { WW_OFF = 0, WW_LINEAR = 1, WW_MLP = 2 };
constexpr int WW_MAX_DEPTH = 64;
constexpr int IMP_MAX_NX = 256, IMP_MAX_NE = 64;
constexpr uint16_t IV_EMPTY = 0x00FF;  // lo 255 > hi 0

struct WwDev {
    int32_t kind;                 // WW_OFF, WW_LINEAR, WW_MLP
    int32_t nmax, depth;          // most copies per split; most pending records per slot
    double lin0, lin1, lin2;      // WW_LINEAR: ln I = lin0 + lin1 f_x + lin2 f_E
    double length, kappa, ratio;  // feature scale L; w_L at the source = 1 / kappa; w_U / w_L
    double ln_emin, ln_erange;    // ln 1e-5 and ln(2e7 / 1e-5)
    double ln_lo, ln_hi;          // ln I clamped to [ln_lo, ln_hi] when ln_lo < ln_hi
    const double *ln_src;         // device scalar: ln I at the source point
    MlpDev mlp;                   // WW_MLP: the network
    uint32_t C;                   // slots
    // pending copies, [level][slot]
    double *sx, *sy, *sz, *su, *sv, *sw, *sE, *swt;
    int32_t *scell, *smat, *sncoll, *sncross;
    uint32_t *slin, *ssplit, *snext, *sn;
    uint8_t *sinside, *sgen;
    uint8_t *depth_of;            // [slot] pending records
    uint32_t *splits;             // [slot] split events of the running copy
    uint8_t *gen;                 // [slot] splits on the running copy's line
    int32_t *inh_coll, *inh_cross;  // [slot] counts the running copy inherited
    // copy bank: Q entries, filled from the stacks, emptied by the refill
    double *qx, *qy, *qz, *qu, *qv, *qw, *qE, *qwt;
    int32_t *qcell, *qmat, *qncoll, *qncross;
    uint8_t *qinside, *qgen;
    uint32_t *qlin;
    uint64_t *qpid;
    uint16_t *qiv;                // [e][Q]
    uint32_t Q;
    // importance estimate (imp_nx == 0: off)
    int32_t imp_nx, imp_ne;
    double imp_x0, imp_x1;
    uint16_t *iv;                 // [e][slot] x-bin interval entered at E-bin e: lo | hi << 8
    uint16_t *siv;                // [level][e][slot] the same for pending copies
    double *num, *den, *cnt;      // [e * nx + x] score credited, weight entered, credits
};

// Lineage of copy k (1..n-1) of split number s of a copy of lineage a: the
// three mixed and run through MurmurHash3's 32-bit finaliser; never 0 (the
// lineage of source particles).
__device__ __forceinline__ uint32_t child_lineage(uint32_t a, uint32_t s, uint32_t k)
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

// ---------------------------------------------------------------------------
// importance estimate
// ---------------------------------------------------------------------------
__device__ __forceinline__ int32_t imp_xbin(const WwDev &W, double x)
{
    const double t = floor((x - W.imp_x0) / (W.imp_x1 - W.imp_x0) * W.imp_nx);
    if (!(t > 0.0)) return 0;
    return t > (double)(W.imp_nx - 1) ? W.imp_nx - 1 : (int32_t)t;
}

__device__ __forceinline__ int32_t imp_ebin(const WwDev &W, double E)
{
    const double t = floor((log(E) - W.ln_emin) / W.ln_erange * W.imp_ne);
    if (!(t > 0.0)) return 0;
    return t > (double)(W.imp_ne - 1) ? W.imp_ne - 1 : (int32_t)t;
}

// The copy in slot s moved from x = xa to x = xb at energy E with weight w:
// mark the cells passed, adding w to the denominator of each cell it enters
// for the first time.
__device__ inline void imp_enter(const WwDev &W, uint32_t s, double xa, double xb, double E, double w)
{
    const int32_t e = imp_ebin(W, E);
    int32_t a = imp_xbin(W, xa), b = imp_xbin(W, xb);
    if (a > b) {
        const int32_t t = a;
        a = b;
        b = t;
    }
    uint16_t *slot = W.iv + (size_t)e * W.C + s;
    const uint16_t v = *slot;
    int32_t lo = v & 0xFF, hi = v >> 8;
    double *den = W.den + (size_t)e * W.imp_nx;
    if (lo > hi) {
        for (int32_t g = a; g <= b; ++g) atomicAdd(den + g, w);
        lo = a;
        hi = b;
    } else {
        for (int32_t g = a; g <= b && g < lo; ++g) atomicAdd(den + g, w);
        for (int32_t g = (a > hi + 1 ? a : hi + 1); g <= b; ++g) atomicAdd(den + g, w);
        lo = a < lo ? a : lo;
        hi = b > hi ? b : hi;
    }
    *slot = (uint16_t)(lo | (hi << 8));
}

// A score w: credit every cell the copy in slot s has entered.
__device__ inline void imp_credit(const WwDev &W, uint32_t s, double w)
{
    for (int32_t e = 0; e < W.imp_ne; ++e) {
        const uint16_t v = W.iv[(size_t)e * W.C + s];
        const int32_t lo = v & 0xFF, hi = v >> 8;
        for (int32_t g = lo; g <= hi; ++g) {
            atomicAdd(W.num + (size_t)e * W.imp_nx + g, w);
            atomicAdd(W.cnt + (size_t)e * W.imp_nx + g, 1.0);
        }
    }
}

// A new source particle in slot s: nothing pending, no cells entered but the
// source point's.
__device__ inline void ww_start(const WwDev &W, uint32_t s, double x, double E)
{
    if (W.depth_of) {
        W.depth_of[s] = 0;
        W.splits[s] = 0;
        W.gen[s] = 0;
        W.inh_coll[s] = 0;
        W.inh_cross[s] = 0;
    }
    if (W.imp_nx) {
        for (int32_t e = 0; e < W.imp_ne; ++e) W.iv[(size_t)e * W.C + s] = IV_EMPTY;
        imp_enter(W, s, x, x, E, 1.0);
    }
}

// ---------------------------------------------------------------------------
// weight windows
// ---------------------------------------------------------------------------
__device__ __forceinline__ double ww_ln_importance_linear(const WwDev &W, const Particle &p)
{
    const double fx = p.x / W.length;
    const double fe = (log(p.E) - W.ln_emin) / W.ln_erange;
    return W.lin0 + W.lin1 * fx + W.lin2 * fe;
}

// ln I of the particles of a workgroup.  WW_MLP: the network, one sample per
// lane, on the matrix cores -- every thread of the workgroup must call it
// (lanes with chk false pass zeros and get a value to ignore).
__device__ __forceinline__ double ww_clamp(const WwDev &W, double v)
{
    return W.ln_lo < W.ln_hi ? fmin(fmax(v, W.ln_lo), W.ln_hi) : v;
}

template <int WWK>
__device__ inline double ww_ln_importance(const WwDev &W, const Particle &p, bool chk)
{
    if constexpr (WWK == WW_LINEAR) {
        return chk ? ww_clamp(W, ww_ln_importance_linear(W, p)) : 0.0;
    } else {
        __shared__ __attribute__((aligned(16))) uint16_t h1s[WAVES][64 * H1_STRIDE];
        __shared__ float ys[WAVES][64];
        if (!__syncthreads_or(chk)) return 0.0;
        float f[4] = {0.f, 0.f, 0.f, 0.f};
        if (chk) mlp_features(p.x, p.y, p.z, p.E, W.length, W.ln_emin, W.ln_erange, f);
        const int wave = threadIdx.x >> 6;
        return ww_clamp(W, (double)wave_mlp(W.mlp, f, h1s[wave], ys[wave]));
    }
}

__device__ inline void ww_push(const WwDev &W, uint32_t s, const Particle &p, uint32_t n)
{
    const uint32_t d = W.depth_of[s];
    const size_t k = (size_t)d * W.C + s;
    W.sx[k] = p.x; W.sy[k] = p.y; W.sz[k] = p.z;
    W.su[k] = p.u; W.sv[k] = p.v; W.sw[k] = p.w;
    W.sE[k] = p.E; W.swt[k] = p.wt;
    W.scell[k] = p.cell; W.smat[k] = p.mat; W.sinside[k] = p.inside ? 1 : 0;
    W.sncoll[k] = p.ncoll; W.sncross[k] = p.ncross;
    W.slin[k] = p.lineage; W.ssplit[k] = W.splits[s]; W.snext[k] = 1u; W.sn[k] = n;
    W.sgen[k] = W.gen[s];
    if (W.imp_nx) {
        for (int32_t e = 0; e < W.imp_ne; ++e)
            W.siv[((size_t)d * W.imp_ne + e) * W.C + s] = W.iv[(size_t)e * W.C + s];
    }
    W.depth_of[s] = (uint8_t)(d + 1);
    W.splits[s] += 1u;
}

// Window check of the copy in slot s at its point, ln I given.  Returns
// FATE_ROULETTE when roulette kills it, else 0 (a split leaves the copy that
// goes on in p and pushes the others).
__device__ inline int32_t ww_check(const WwDev &W, uint32_t s, Particle &p, double ln_i, uint64_t seed,
                                   StepScore &sc)
{
    const double lw = exp(*W.ln_src - ln_i) / W.kappa;
    const double uw = W.ratio * lw;
    const double sw = 0.5 * (lw + uw);
    const double w = p.wt;
    if (w > uw) {
        const double nd = ceil(w / uw);
        const int32_t n = nd > (double)W.nmax ? W.nmax : (int32_t)nd;
        if (n >= 2 && (int32_t)W.gen[s] < W.depth) {
            p.wt = w / (double)n;
            W.gen[s] += 1;  // the copy that goes on and its n - 1 siblings
            ww_push(W, s, p, (uint32_t)n);
            sc.g[G_SPLIT] += (double)(n - 1);
        }
        return 0;
    }
    if (w < lw) {
        Rng rng(seed, p.pid, p.lineage, p.ndraw);
        const double xi = rng.next();
        p.ndraw = rng.n;
        if (xi < w / sw) {
            p.wt = sw;
            return 0;
        }
        sc.g[G_ROULETTE] += 1.0;
        return FATE_ROULETTE;
    }
    return 0;
}

// The copy in p (slot s) has died and the slot has a pending copy: take the
// next one off the stack into p.  Its state is the parent's at the split, its
// stream the child lineage's from draw 0, its path length starts at 0.
__device__ inline void ww_pop(const WwDev &W, uint32_t s, Particle &p)
{
    const uint32_t d = (uint32_t)W.depth_of[s] - 1u;
    const size_t k = (size_t)d * W.C + s;
    const uint32_t kk = W.snext[k], n = W.sn[k];
    W.inh_coll[s] = W.sncoll[k];
    W.inh_cross[s] = W.sncross[k];
    W.gen[s] = W.sgen[k];
    p.track = 0.0;
    p.x = W.sx[k]; p.y = W.sy[k]; p.z = W.sz[k];
    p.u = W.su[k]; p.v = W.sv[k]; p.w = W.sw[k];
    p.E = W.sE[k]; p.wt = W.swt[k];
    p.cell = W.scell[k]; p.mat = W.smat[k]; p.inside = W.sinside[k] != 0;
    p.ncoll = W.sncoll[k]; p.ncross = W.sncross[k];
    p.lineage = child_lineage(W.slin[k], W.ssplit[k], kk);
    p.ndraw = 0u;
    W.splits[s] = 0u;
    if (W.imp_nx) {
        for (int32_t e = 0; e < W.imp_ne; ++e)
            W.iv[(size_t)e * W.C + s] = W.siv[((size_t)d * W.imp_ne + e) * W.C + s];
    }
    if (kk + 1u >= n) W.depth_of[s] = (uint8_t)d;
    else W.snext[k] = kk + 1u;
}

__device__ __forceinline__ bool ww_pending(const WwDev &W, uint32_t s) { return W.depth_of && W.depth_of[s] > 0; }

// History record of a copy that ended: its collisions, crossings, draws and
// path length add to its history's (the record starts zeroed; copies of one
// history may end in any order and in parallel); the source particle's own
// copy (lineage 0) also sets the fate, final energy and weight.
__device__ __forceinline__ void log_copy(HistLog *log, uint64_t first_pid, const Particle &p, int32_t fate,
                                         const WwDev &W, uint32_t s)
{
    HistLog *h = log + (p.pid - first_pid);
    atomicAdd(&h->n_coll, p.ncoll - W.inh_coll[s]);
    atomicAdd(&h->n_cross, p.ncross - W.inh_cross[s]);
    atomicAdd(reinterpret_cast<unsigned long long *>(&h->n_draws), (unsigned long long)p.ndraw);
    atomicAdd(&h->track, p.track);
    if (p.lineage == 0u) {
        h->fate = fate;
        h->E_final = p.E;
        h->weight = p.wt;
    }
}

// Pending copies in the stack of slot s.
__device__ __forceinline__ uint32_t ww_pending_copies(const WwDev &W, uint32_t s)
{
    uint32_t c = 0;
    const uint32_t depth = W.depth_of[s] < (uint32_t)W.depth ? W.depth_of[s] : (uint32_t)W.depth;
    for (uint32_t d = 0; d < depth; ++d) {
        const size_t k = (size_t)d * W.C + s;
        c += W.sn[k] - W.snext[k];
    }
    return c;
}

// Move the pending copies of slot s (pid `pid`) into the copy bank at q0..;
// the stack ends empty.
__device__ inline void ww_flush_slot(const WwDev &W, uint32_t s, uint64_t pid, uint32_t q0)
{
    uint32_t q = q0;
    const uint32_t depth = W.depth_of[s] < (uint32_t)W.depth ? W.depth_of[s] : (uint32_t)W.depth;
    for (uint32_t d = 0; d < depth; ++d) {
        const size_t k = (size_t)d * W.C + s;
        for (uint32_t kk = W.snext[k]; kk < W.sn[k]; ++kk, ++q) {
            W.qx[q] = W.sx[k]; W.qy[q] = W.sy[k]; W.qz[q] = W.sz[k];
            W.qu[q] = W.su[k]; W.qv[q] = W.sv[k]; W.qw[q] = W.sw[k];
            W.qE[q] = W.sE[k]; W.qwt[q] = W.swt[k];
            W.qcell[q] = W.scell[k]; W.qmat[q] = W.smat[k]; W.qinside[q] = W.sinside[k];
            W.qncoll[q] = W.sncoll[k]; W.qncross[q] = W.sncross[k];
            W.qgen[q] = W.sgen[k];
            W.qlin[q] = child_lineage(W.slin[k], W.ssplit[k], kk);
            W.qpid[q] = pid;
            if (W.imp_nx) {
                for (int32_t e = 0; e < W.imp_ne; ++e)
                    W.qiv[(size_t)e * W.Q + q] = W.siv[((size_t)d * W.imp_ne + e) * W.C + s];
            }
        }
    }
    W.depth_of[s] = 0;
}

}  // namespace mc
