"""CPU oracle for the Monte Carlo transport hot path -- TEST INFRASTRUCTURE.

Only the test-suite, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  The GPU library never loads it
and shares no code with it; both read the same synthetic inputs made by
``mcsynth``.

The arithmetic lives in ``oracle.c`` (plain C, fp64, -ffp-contract=off), built
here into ``liboracle.so`` with gcc; this module only marshals arguments and
forms batch statistics.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# global tally slots (see oracle.c)
G_TRACK, G_COLL_EST, G_ABSORB, G_CUTOFF, G_LEAK, G_TRACK_ABS = 0, 1, 2, 3, 4, 5
G_NCOLL, G_NCROSS, G_LEAK_XHI, G_LEAK_XHI_UNC, G_SPLIT, G_ROULETTE, N_GLOBAL = 6, 7, 8, 9, 10, 11, 12
FATE_ABSORBED, FATE_CUTOFF, FATE_LEAKED, FATE_LOST, FATE_ROULETTE = 1, 2, 3, 4, 5


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (-O2 -fopenmp -ffp-contract=off)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared",
                               "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-Wall",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Problem(C.Structure):
    _fields_ = [
        ("n_nuc", C.c_int32), ("nuc_off", C.POINTER(C.c_int64)),
        ("E", C.POINTER(C.c_double)), ("sig_c", C.POINTER(C.c_double)),
        ("sig_s", C.POINTER(C.c_double)), ("awr", C.POINTER(C.c_double)),
        ("n_mat", C.c_int32), ("mat_off", C.POINTER(C.c_int32)),
        ("mat_nuc", C.POINTER(C.c_int32)), ("mat_dens", C.POINTER(C.c_double)),
        ("geom_kind", C.c_int32), ("inf_material", C.c_int32),
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("pitch", C.c_double), ("radius", C.c_double), ("z0", C.c_double), ("z1", C.c_double),
        ("pin_mat", C.POINTER(C.c_int32)), ("mod_mat", C.c_int32), ("bc", C.c_int32 * 6),
        ("n_layers", C.c_int32), ("x_edges", C.POINTER(C.c_double)),
        ("layer_mat", C.POINTER(C.c_int32)),
        ("src_kind", C.c_int32), ("src_pos", C.c_double * 3), ("src_box", C.c_double * 6),
        ("src_dir", C.c_double * 3), ("src_E", C.c_double),
        ("tally_kind", C.c_int32), ("n_ebins", C.c_int32), ("e_edges", C.POINTER(C.c_double)),
        ("mesh_dims", C.c_int32 * 3), ("mesh_box", C.c_double * 6),
        ("e_cut", C.c_double), ("max_events", C.c_int64),
        ("ww_kind", C.c_int32), ("ww_lin", C.c_double * 3), ("ww_mlp", C.POINTER(C.c_double)),
        ("ww_length", C.c_double), ("ww_kappa", C.c_double), ("ww_ratio", C.c_double),
        ("ww_nmax", C.c_int32), ("ww_depth", C.c_int32),
        ("imp_nx", C.c_int32), ("imp_ne", C.c_int32), ("imp_x0", C.c_double), ("imp_x1", C.c_double),
        ("ww_ln_lo", C.c_double), ("ww_ln_hi", C.c_double),
        ("n_chan", C.c_int32), ("chan", C.POINTER(C.c_double)),
    ]


class _History(C.Structure):
    _fields_ = [("fate", C.c_int32), ("n_coll", C.c_int32), ("n_cross", C.c_int32),
                ("pad", C.c_int32), ("n_draws", C.c_uint64), ("E_final", C.c_double),
                ("track", C.c_double), ("weight", C.c_double)]


HISTORY_DTYPE = np.dtype([("fate", np.int32), ("n_coll", np.int32), ("n_cross", np.int32),
                          ("pad", np.int32), ("n_draws", np.uint64), ("E_final", np.float64),
                          ("track", np.float64), ("weight", np.float64)])

_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        D, P = C.c_double, C.POINTER
        _lib.orc_philox4x32_10.argtypes = [P(C.c_uint32), P(C.c_uint32), P(C.c_uint32)]
        _lib.orc_uniform.argtypes = [C.c_uint64, C.c_uint32, C.c_uint64, C.c_uint64]
        _lib.orc_uniform.restype = D
        _lib.orc_grid_index.argtypes = [P(D), C.c_int64, D]
        _lib.orc_grid_index.restype = C.c_int64
        _lib.orc_micro_xs.argtypes = [P(_Problem), C.c_int32, D, P(D), P(D), P(C.c_int64)]
        _lib.orc_macro_xs.argtypes = [P(_Problem), C.c_int32, D, P(D), P(D)]
        _lib.orc_elastic.argtypes = [D, D, D, P(D), P(D)]
        _lib.orc_rotate.argtypes = [P(D), D, D]
        _lib.orc_run.argtypes = [P(_Problem), C.c_uint64, C.c_uint64, C.c_uint64, P(D), P(D),
                                 P(D), C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]
        _lib.orc_bf16.argtypes = [D]
        _lib.orc_bf16.restype = D
        _lib.orc_mlp_forward.argtypes = [P(D), P(D)]
        _lib.orc_mlp_forward.restype = D
        _lib.orc_child_lineage.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32]
        _lib.orc_child_lineage.restype = C.c_uint32
        _lib.orc_ln_importance_source.argtypes = [P(_Problem)]
        _lib.orc_ln_importance_source.restype = D
        _lib.orc_run.restype = C.c_int
        _lib.orc_run_scatter_stats.argtypes = [P(_Problem), C.c_uint64, C.c_uint64, C.c_uint64, P(D), C.c_int]
        _lib.orc_run_scatter_stats.restype = C.c_int
        _lib.orc_max_threads.restype = C.c_int
        _lib.orc_micro_xs_many.argtypes = [P(_Problem), C.c_int32, C.c_int64, P(D), P(C.c_int64), P(D), P(D)]
        _lib.orc_macro_xs_many.argtypes = [P(_Problem), C.c_int64, P(C.c_int32), P(D), P(D), P(D)]
        _lib.orc_macro_channels_many.argtypes = [P(_Problem), C.c_int64, P(C.c_int32), P(D), P(D)]
        _lib.orc_faddeeva_init.argtypes = []
        _lib.orc_faddeeva_many.argtypes = [C.c_int64, P(D), P(D), P(D), P(D)]
        _lib.orc_faddeeva_coeffs.argtypes = [P(D), P(D)]
        _lib.orc_mp_macro_many.argtypes = [P(_MpNuclide), P(D), C.c_int32, P(C.c_int32), P(D), D, C.c_int64,
                                           P(D), P(D), P(D)]
        _lib.orc_faddeeva_init()
    return _lib


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class _MpNuclide(C.Structure):
    _fields_ = [("n_poles", C.c_int32), ("n_windows", C.c_int32), ("n_bg", C.c_int32), ("pad", C.c_int32),
                ("u_lo", C.c_double), ("u_hi", C.c_double),
                ("poles", C.POINTER(C.c_double)), ("res_c", C.POINTER(C.c_double)),
                ("res_s", C.POINTER(C.c_double)), ("win", C.POINTER(C.c_int32)),
                ("bg_c", C.POINTER(C.c_double)), ("bg_s", C.POINTER(C.c_double))]


def _iptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


class OracleProblem:
    """Flattened arrays of a ``mcsynth.Problem`` held alive for the C structure."""

    def __init__(self, prob, max_events: int = 10_000_000):
        self.prob = prob
        nucs = prob.nuclides
        lens = np.array([n.E.size for n in nucs], np.int64)
        self.nuc_off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
        self.E = np.ascontiguousarray(np.concatenate([n.E for n in nucs]), np.float64)
        self.sc = np.ascontiguousarray(np.concatenate([n.sig_c for n in nucs]), np.float64)
        self.ss = np.ascontiguousarray(np.concatenate([n.sig_s for n in nucs]), np.float64)
        self.awr = np.array([n.awr for n in nucs], np.float64)
        mats = prob.materials
        self.mat_off = np.concatenate([[0], np.cumsum([m.nuclides.size for m in mats])]).astype(np.int32)
        self.mat_nuc = np.ascontiguousarray(np.concatenate([m.nuclides for m in mats]), np.int32)
        self.mat_dens = np.ascontiguousarray(np.concatenate([m.densities for m in mats]), np.float64)
        g, s, t = prob.geometry, prob.source, prob.tally
        self.pin_mat = np.ascontiguousarray(g.pin_material if g.pin_material is not None
                                            else np.zeros(1, np.int32), np.int32)
        self.x_edges = np.ascontiguousarray(g.x_edges if g.x_edges is not None
                                            else np.zeros(2), np.float64)
        self.layer_mat = np.ascontiguousarray(g.layer_material if g.layer_material is not None
                                              else np.zeros(1, np.int32), np.int32)
        self.e_edges = np.ascontiguousarray(t.energy_edges if t.energy_edges is not None
                                            else np.zeros(2), np.float64)
        c = _Problem()
        c.n_nuc = len(nucs)
        c.nuc_off = self.nuc_off.ctypes.data_as(C.POINTER(C.c_int64))
        c.E, c.sig_c, c.sig_s, c.awr = _dptr(self.E), _dptr(self.sc), _dptr(self.ss), _dptr(self.awr)
        c.n_mat = len(mats)
        c.mat_off, c.mat_nuc, c.mat_dens = _iptr(self.mat_off), _iptr(self.mat_nuc), _dptr(self.mat_dens)
        c.geom_kind, c.inf_material = g.kind, g.material
        c.nx, c.ny, c.pitch, c.radius, c.z0, c.z1 = g.nx, g.ny, g.pitch, g.radius, g.z0, g.z1
        c.pin_mat, c.mod_mat = _iptr(self.pin_mat), g.moderator_material
        c.bc = (C.c_int32 * 6)(*g.bc)
        c.n_layers = 0 if g.x_edges is None else len(g.x_edges) - 1
        c.x_edges, c.layer_mat = _dptr(self.x_edges), _iptr(self.layer_mat)
        c.src_kind = s.kind
        c.src_pos = (C.c_double * 3)(*s.position)
        c.src_box = (C.c_double * 6)(*s.box)
        c.src_dir = (C.c_double * 3)(*s.direction)
        c.src_E = s.energy
        c.tally_kind = t.kind
        c.n_ebins = 0 if t.energy_edges is None else len(t.energy_edges) - 1
        c.e_edges = _dptr(self.e_edges)
        c.mesh_dims = (C.c_int32 * 3)(*t.mesh_dims)
        c.mesh_box = (C.c_double * 6)(*t.mesh_box)
        c.e_cut = prob.energy_cutoff
        c.max_events = max_events
        ww = prob.ww
        c.ww_kind = ww.kind
        c.ww_lin = (C.c_double * 3)(*ww.lin)
        self.ww_mlp = np.ascontiguousarray(ww.mlp if ww.mlp is not None else np.zeros(4545), np.float64)
        c.ww_mlp = _dptr(self.ww_mlp)
        c.ww_length, c.ww_kappa, c.ww_ratio = ww.length, ww.kappa, ww.ratio
        c.ww_nmax, c.ww_depth = ww.n_max, ww.depth
        c.ww_ln_lo, c.ww_ln_hi = ww.ln_lo, ww.ln_hi
        c.imp_nx, c.imp_ne, c.imp_x0, c.imp_x1 = prob.imp.nx, prob.imp.ne, prob.imp.x0, prob.imp.x1
        chans = getattr(prob, "channels", None)
        self.n_chan = 0 if not chans else int(chans[0].shape[1])
        if self.n_chan:
            assert all(ch.shape == (n.E.size, self.n_chan) for ch, n in zip(chans, nucs))
            self.chan = np.ascontiguousarray(np.concatenate(chans, axis=0), np.float64)
        else:
            self.chan = np.zeros(1)
        c.n_chan = self.n_chan
        c.chan = _dptr(self.chan)
        self.n_mat = len(mats)
        self.n_nuc = len(nucs)
        self.c = c
        self.n_cells = prob.imp.cells
        self.n_bins = prob.n_bins

    def ref(self):
        return C.byref(self.c)


# ------------------------------------------------------------------------
# thin wrappers
# ------------------------------------------------------------------------

def philox4x32_10(ctr, key):
    L = lib()
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (C.c_uint32 * 4)()
    L.orc_philox4x32_10(c, k, o)
    return [int(x) for x in o]


def uniform(seed: int, lineage: int, pid: int, n: int) -> float:
    return lib().orc_uniform(seed, lineage, pid, n)


def grid_index(grid: np.ndarray, e: float) -> int:
    g = np.ascontiguousarray(grid, np.float64)
    return int(lib().orc_grid_index(_dptr(g), g.size, float(e)))


def micro_xs(op: OracleProblem, nuc: int, energies):
    """(grid index, sigma_c, sigma_s) of nuclide ``nuc`` at each energy."""
    e = np.ascontiguousarray(energies, np.float64).ravel()
    sc = np.empty(e.size)
    ss = np.empty(e.size)
    idx = np.empty(e.size, np.int64)
    lib().orc_micro_xs_many(op.ref(), nuc, e.size, _dptr(e), idx.ctypes.data_as(C.POINTER(C.c_int64)),
                            _dptr(sc), _dptr(ss))
    return idx, sc, ss


def macro_xs(op: OracleProblem, mats, energies):
    """(Sigma_a, Sigma_s) of each (material, energy) pair."""
    e = np.ascontiguousarray(energies, np.float64).ravel()
    m = np.ascontiguousarray(np.broadcast_to(np.asarray(mats, np.int32), np.shape(energies)), np.int32).ravel()
    Sa = np.empty(e.size)
    Ss = np.empty(e.size)
    lib().orc_macro_xs_many(op.ref(), e.size, _iptr(m), _dptr(e), _dptr(Sa), _dptr(Ss))
    return Sa, Ss


def macro_channels(op: OracleProblem, mats, energies):
    """[n, n_chan] macroscopic reaction-channel cross sections of each
    (material, energy) pair."""
    e = np.ascontiguousarray(energies, np.float64).ravel()
    m = np.ascontiguousarray(np.broadcast_to(np.asarray(mats, np.int32), np.shape(energies)), np.int32).ravel()
    out = np.empty((e.size, op.n_chan))
    lib().orc_macro_channels_many(op.ref(), e.size, _iptr(m), _dptr(e), _dptr(out))
    return out


def faddeeva(z):
    """w(z) for Im z > 0 (the oracle's rational series)."""
    z = np.ascontiguousarray(np.asarray(z, np.complex128).ravel())
    zr, zi = np.ascontiguousarray(z.real), np.ascontiguousarray(z.imag)
    wr, wi = np.empty(z.size), np.empty(z.size)
    lib().orc_faddeeva_many(z.size, _dptr(zr), _dptr(zi), _dptr(wr), _dptr(wi))
    return wr + 1j * wi


def faddeeva_coeffs():
    """(L, a[0..N-1]) of the oracle's rational series for w(z): the constants a
    rounding bound of a pole term needs."""
    L = C.c_double()
    a = np.empty(32)
    lib().orc_faddeeva_coeffs(C.byref(L), _dptr(a))
    return float(L.value), a


def multipole_macro(nucs, mat_ids, dens, T: float, energies):
    """(Sigma_a, Sigma_s) of a material of multipole nuclides (a list of
    mcsynth.MultipoleNuclide; the material's ids and densities) at temperature
    T (K) for each energy."""
    keep = []

    def arr(a, dt):
        a = np.ascontiguousarray(a, dt)
        keep.append(a)
        return a

    cs = (_MpNuclide * len(nucs))()
    for c, nd in zip(cs, nucs):
        c.n_poles, c.n_windows, c.n_bg = nd.poles.size, nd.win.shape[0], nd.bg_c.shape[1]
        c.u_lo, c.u_hi = nd.u_lo, nd.u_hi
        c.poles = _dptr(arr(nd.poles.view(np.float64), np.float64))
        c.res_c = _dptr(arr(nd.res_c.view(np.float64), np.float64))
        c.res_s = _dptr(arr(nd.res_s.view(np.float64), np.float64))
        c.win = _iptr(arr(nd.win, np.int32))
        c.bg_c = _dptr(arr(nd.bg_c, np.float64))
        c.bg_s = _dptr(arr(nd.bg_s, np.float64))
    awr = arr([nd.awr for nd in nucs], np.float64)
    ids = arr(mat_ids, np.int32)
    d = arr(dens, np.float64)
    e = arr(np.ravel(energies), np.float64)
    Sa, Ss = np.empty(e.size), np.empty(e.size)
    lib().orc_mp_macro_many(cs, _dptr(awr), ids.size, _iptr(ids), _dptr(d), float(T), e.size, _dptr(e),
                            _dptr(Sa), _dptr(Ss))
    return Sa, Ss


def elastic(A: float, E: float, mu_cm: float):
    a, b = C.c_double(), C.c_double()
    lib().orc_elastic(A, E, mu_cm, C.byref(a), C.byref(b))
    return a.value, b.value


def rotate(d, mu: float, phi: float):
    arr = (C.c_double * 3)(*d)
    lib().orc_rotate(arr, mu, phi)
    return np.array(list(arr))


@dataclass
class RunResult:
    n: int
    tl: np.ndarray       # raw track-length sums per bin
    coll: np.ndarray     # raw collision-estimator sums per bin
    glob: np.ndarray     # raw global sums (N_GLOBAL)
    history: np.ndarray | None = None
    imp: np.ndarray | None = None   # [3, cells]: score credited, weight entered, credits
    rr: np.ndarray | None = None    # [n_mat, n_chan] raw track-length reaction rates


def run(op: OracleProblem, seed: int, first_pid: int, n: int, history: bool = False,
        threads: int = 0) -> RunResult:
    """Track histories [first_pid, first_pid + n) birth to death; raw sums."""
    nb = op.n_bins
    tl = np.zeros(nb)
    coll = np.zeros(nb)
    glob = np.zeros(N_GLOBAL)
    imp = np.zeros(3 * op.n_cells) if op.n_cells else None
    hist = np.zeros(n, HISTORY_DTYPE) if history else None
    rr = np.zeros(op.n_mat * op.n_chan) if op.n_chan else None
    rc = lib().orc_run(op.ref(), seed, first_pid, n, _dptr(tl), _dptr(coll), _dptr(glob),
                       imp.ctypes.data if imp is not None else None,
                       rr.ctypes.data if rr is not None else None,
                       hist.ctypes.data if history else None, threads)
    if rc != 0:
        raise MemoryError("oracle run failed")
    return RunResult(n=n, tl=tl, coll=coll, glob=glob, history=hist,
                     imp=imp.reshape(3, -1) if imp is not None else None,
                     rr=rr.reshape(op.n_mat, op.n_chan) if rr is not None else None)


def scatter_stats(op: OracleProblem, seed: int, first_pid: int, n: int, threads: int = 0) -> np.ndarray:
    """Per target nuclide k of the collisions of histories [first_pid,
    first_pid + n): row k = (scatterings on k, sum of ln(E / E') over them).
    Test statistics of the target selection; the tallies are discarded."""
    ns = np.zeros(2 * op.n_nuc)
    rc = lib().orc_run_scatter_stats(op.ref(), seed, first_pid, n, _dptr(ns), threads)
    if rc != 0:
        raise MemoryError("oracle run failed")
    return ns.reshape(-1, 2)


def bf16(x: float) -> float:
    return float(lib().orc_bf16(float(x)))


def mlp_forward(params: np.ndarray, f) -> float:
    p = np.ascontiguousarray(params, np.float64)
    ff = np.ascontiguousarray(f, np.float64)
    return float(lib().orc_mlp_forward(_dptr(p), _dptr(ff)))


def child_lineage(a: int, s: int, k: int) -> int:
    return int(lib().orc_child_lineage(a, s, k))


def ln_importance_source(op: OracleProblem) -> float:
    return float(lib().orc_ln_importance_source(op.ref()))


IMP_SAMPLE_LINEAGE = 0x5EED0002


def importance_samples(num, den, cnt, nx: int, ne: int, x0: float, x1: float, length: float, replicas: int,
                       min_credits: float, rel_floor: float, seed: int):
    """Training samples of the importance network from forward importance sums
    (cells e * nx + x, in index order).  A cell with at least ``min_credits``
    detector credits and positive sums gives ``replicas`` samples: features
    (x centre / length, f_y, f_z, (e + 1/2) / ne) with f_y, f_z = 2u - 1 from
    draws 2r and 2r + 1 of the Philox stream (seed, pid = cell, lineage
    IMP_SAMPLE_LINEAGE), target ln(num / den) (the forward estimate of the
    importance), weight 1 / (1 / cnt + rel_floor^2) (its inverse relative
    variance, floored).  Returns float32 arrays X [n, 4], T [n], W [n]."""
    X, T, W = [], [], []
    for g in range(nx * ne):
        if not (cnt[g] >= min_credits and num[g] > 0.0 and den[g] > 0.0):
            continue
        ix, e = g % nx, g // nx
        xc = x0 + (x1 - x0) * (ix + 0.5) / nx
        fx = np.float32(xc / length)
        fe = np.float32((e + 0.5) / ne)
        tg = np.float32(math.log(num[g] / den[g]))
        wt = np.float32(1.0 / (1.0 / cnt[g] + rel_floor * rel_floor))
        for r in range(replicas):
            uy = uniform(seed, IMP_SAMPLE_LINEAGE, g, 2 * r)
            uz = uniform(seed, IMP_SAMPLE_LINEAGE, g, 2 * r + 1)
            X.append([fx, np.float32(2.0 * uy - 1.0), np.float32(2.0 * uz - 1.0), fe])
            T.append(tg)
            W.append(wt)
    return (np.array(X, np.float32).reshape(-1, 4), np.array(T, np.float32), np.array(W, np.float32))


@dataclass
class BatchStats:
    mean: dict
    stderr: dict
    n_batches: int


def run_batches(op: OracleProblem, seed: int, n_batches: int, per_batch: int,
                first_pid: int = 0, threads: int = 0) -> BatchStats:
    """Batch statistics: each batch's per-source-particle tally T_b; mean = S1/B,
    standard error = sqrt((S2/B - mean^2) / (B - 1))."""
    acc = {k: [0.0, 0.0] for k in ("tl", "coll", "glob") + (("rr",) if op.n_chan else ())}
    for b in range(n_batches):
        r = run(op, seed, first_pid + b * per_batch, per_batch, threads=threads)
        for k in acc:
            T = getattr(r, k) / per_batch
            acc[k][0] = acc[k][0] + T
            acc[k][1] = acc[k][1] + T * T
    mean, se = {}, {}
    B = n_batches
    for k, (s1, s2) in acc.items():
        m = s1 / B
        mean[k] = m
        se[k] = np.sqrt(np.maximum(s2 / B - m * m, 0.0) / max(B - 1, 1))
    return BatchStats(mean=mean, stderr=se, n_batches=B)


def max_threads() -> int:
    return int(lib().orc_max_threads())
