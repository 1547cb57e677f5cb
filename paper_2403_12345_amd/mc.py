"""Thin ctypes binding of libmc.so (declarations in include/mc.h).

Every function here has the name of the C entry point it calls and only
marshals arguments: numpy arrays for host inputs, torch tensors (or raw
integers) for device pointers, torch's current HIP stream for the stream.
Every step of the transport path runs in the library's HIP kernels; there is
no Python or CPU fallback.  Loading fails loudly when libmc.so is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmc.so")

MC_OK, MC_EINVAL, MC_ENOMEM, MC_EHIP, MC_ELOST, MC_ESTATE, MC_ENODEV, MC_ERANGE = 0, -1, -2, -3, -4, -5, -6, -7
MC_GEOM_INFINITE, MC_GEOM_LATTICE, MC_GEOM_SLAB = 0, 1, 2
MC_TALLY_ENERGY, MC_TALLY_PIN, MC_TALLY_MESH, MC_TALLY_SLAB = 0, 1, 2, 3
MC_T_FLUX_TRACK, MC_T_FLUX_COLLISION, MC_T_GLOBAL, MC_T_REACTION = 0, 1, 2, 3
MC_MAX_CHANNELS = 16
(MC_G_TRACK, MC_G_COLL_EST, MC_G_ABSORB, MC_G_CUTOFF, MC_G_LEAK, MC_G_TRACK_ABS, MC_G_NCOLL,
 MC_G_NCROSS, MC_G_LEAK_XHI, MC_G_LEAK_XHI_UNC, MC_G_SPLIT, MC_G_ROULETTE, MC_N_GLOBAL) = range(13)
MC_FATE_ABSORBED, MC_FATE_CUTOFF, MC_FATE_LEAKED, MC_FATE_LOST, MC_FATE_ROULETTE = 1, 2, 3, 4, 5
MC_WW_OFF, MC_WW_LINEAR, MC_WW_MLP = 0, 1, 2

_STATUS = {MC_EINVAL: "MC_EINVAL", MC_ENOMEM: "MC_ENOMEM", MC_EHIP: "MC_EHIP", MC_ELOST: "MC_ELOST",
           MC_ESTATE: "MC_ESTATE", MC_ENODEV: "MC_ENODEV", MC_ERANGE: "MC_ERANGE"}


class MCError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


class mc_geometry_desc(C.Structure):
    _fields_ = [
        ("kind", C.c_int32), ("material", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32),
        ("pitch", C.c_double), ("radius", C.c_double), ("z0", C.c_double), ("z1", C.c_double),
        ("pin_material", C.POINTER(C.c_int32)), ("moderator_material", C.c_int32),
        ("bc", C.c_int32 * 6), ("n_layers", C.c_int32), ("x_edges", C.POINTER(C.c_double)),
        ("layer_material", C.POINTER(C.c_int32)), ("source_kind", C.c_int32),
        ("source_pos", C.c_double * 3), ("source_box", C.c_double * 6),
        ("source_dir", C.c_double * 3), ("source_energy", C.c_double),
        ("tally_kind", C.c_int32), ("n_energy_bins", C.c_int32),
        ("energy_edges", C.POINTER(C.c_double)), ("mesh_dims", C.c_int32 * 3),
        ("mesh_box", C.c_double * 6), ("energy_cutoff", C.c_double),
    ]


class mc_run_opts(C.Structure):
    _fields_ = [("in_flight", C.c_uint64), ("sort_min", C.c_uint64), ("no_tally", C.c_int32),
                ("time_kernels", C.c_int32), ("max_events", C.c_int64), ("max_lost", C.c_uint64),
                ("history_log", C.c_void_p)]


class mc_stats(C.Structure):
    _fields_ = [("iterations", C.c_uint64), ("lookups", C.c_uint64), ("nuclide_lookups", C.c_uint64),
                ("lookup_launches", C.c_uint64), ("sorted_lookups", C.c_uint64), ("lost", C.c_uint64),
                ("lookup_bytes", C.c_uint64), ("lookup_ms", C.c_double), ("batch_ms", C.c_double),
                ("tail_particles", C.c_uint64), ("mesh_underflow", C.c_uint64), ("flights", C.c_uint64),
                ("advance_ms", C.c_double), ("cross_ms", C.c_double), ("collide_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class mc_tuning(C.Structure):
    _fields_ = [("lookup_ilp", C.c_int32), ("tail_particles", C.c_int32), ("sort_min", C.c_int32),
                ("in_flight", C.c_int32), ("set_tile_histories", C.c_int32), ("set_grid", C.c_int32),
                ("collide_sort_min", C.c_int32), ("loops", C.c_int32)]
    KEYS = ("lookup_ilp", "tail_particles", "sort_min", "in_flight", "set_tile_histories", "set_grid",
            "collide_sort_min", "loops")

    def as_dict(self):
        return {k: getattr(self, k) for k in self.KEYS}


class mc_problem_desc(C.Structure):
    _fields_ = [("n_nuc", C.c_int32), ("grid_len", C.POINTER(C.c_int32)),
                ("E", C.POINTER(C.POINTER(C.c_double))), ("sig_c", C.POINTER(C.POINTER(C.c_double))),
                ("sig_s", C.POINTER(C.POINTER(C.c_double))), ("awr", C.POINTER(C.c_double)),
                ("n_mat", C.c_int32), ("mat_len", C.POINTER(C.c_int32)), ("mat_nuc", C.POINTER(C.c_int32)),
                ("mat_dens", C.POINTER(C.c_double)), ("geometry", C.POINTER(mc_geometry_desc)),
                ("histories", C.c_uint64), ("seed", C.c_uint64), ("first_pid", C.c_uint64)]


class mc_set_opts(C.Structure):
    _fields_ = [("use_graph", C.c_int32), ("pad", C.c_int32), ("max_events", C.c_int64),
                ("history_log", C.c_void_p)]


class mc_ww_desc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_max", C.c_int32), ("depth", C.c_int32), ("imp_nx", C.c_int32),
                ("imp_ne", C.c_int32), ("reserved", C.c_int32), ("lin", C.c_double * 3), ("length", C.c_double),
                ("kappa", C.c_double), ("ratio", C.c_double), ("imp_x0", C.c_double), ("imp_x1", C.c_double),
                ("ln_lo", C.c_double), ("ln_hi", C.c_double)]


class mc_train_opts(C.Structure):
    _fields_ = [("steps", C.c_int32), ("replicas", C.c_int32), ("lr", C.c_float), ("pad", C.c_float),
                ("min_credits", C.c_double), ("rel_floor", C.c_double), ("length", C.c_double),
                ("seed", C.c_uint64)]


class mc_tally_meta(C.Structure):
    _fields_ = [("n_batches", C.c_uint64), ("n_bins", C.c_uint64), ("histories", C.c_uint64),
                ("s1", C.POINTER(C.c_double)), ("s2", C.POINTER(C.c_double))]


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_void_p)
_RELEASE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p)


class mc_alloc(C.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("release", _RELEASE_FN), ("user", C.c_void_p)]


def _torch_alloc(user, nbytes, device, stream):
    # device memory from PyTorch's caching allocator (NULL -> MC_ENOMEM)
    import torch
    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes), int(device), int(stream or 0))
    except Exception:
        return None


def _torch_release(user, ptr, device, stream):
    import torch
    torch.cuda.caching_allocator_delete(int(ptr))


# one allocator description for every context (the callbacks must outlive them)
_TORCH_ALLOC = mc_alloc(_ALLOC_FN(_torch_alloc), _RELEASE_FN(_torch_release), None)


HISTORY_DTYPE = np.dtype([("fate", np.int32), ("n_coll", np.int32), ("n_cross", np.int32),
                          ("pad", np.int32), ("n_draws", np.uint64), ("E_final", np.float64),
                          ("track", np.float64), ("weight", np.float64)])

_lib = None


def load():
    """Load libmc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it first (python -c 'from paper_2403_12345_amd.build "
                          f"import build_library; build_library()') -- there is no CPU fallback")
    # The library is handed PyTorch's device pointers and streams, so it must
    # run on the HIP runtime PyTorch loaded: load that first.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    P, V, D, I32, U64, SZ = C.POINTER, C.c_void_p, C.c_double, C.c_int32, C.c_uint64, C.c_size_t
    sig = {
        "mc_version": ([], C.c_char_p),
        "mc_create": ([P(V), C.c_int, V, P(mc_alloc)], C.c_int),
        "mc_destroy": ([V], None),
        "mc_last_error": ([V], C.c_char_p),
        "mc_set_stream": ([V, V], C.c_int),
        "mc_init_materials": ([V, I32, P(I32), P(P(D)), P(P(D)), P(P(D)), P(D), I32, P(I32), P(I32),
                               P(D), I32], C.c_int),
        "mc_init_geometry": ([V, P(mc_geometry_desc)], C.c_int),
        "mc_run_batch": ([V, U64, U64, U64, P(mc_run_opts)], C.c_int),
        "mc_run_batches": ([V, U64, U64, U64, U64, P(mc_run_opts)], C.c_int),
        "mc_get_tallies": ([V, I32, P(D), P(D), SZ, P(mc_tally_meta)], C.c_int),
        "mc_set_tallies": ([V, I32, P(D), P(D), SZ, U64, U64], C.c_int),
        "mc_ww_bootstrap_slope": ([V, P(D)], C.c_int),
        "mc_reset_tallies": ([V], C.c_int),
        "mc_get_stats": ([V, P(mc_stats)], C.c_int),
        "mc_lookup_macro": ([V, SZ, V, V, V, V, I32], C.c_int),
        "mc_lookup_macro_noalloc": ([V, SZ, V, V, V, V, I32], C.c_int),
        "mc_init_channels": ([V, I32, P(P(D))], C.c_int),
        "mc_set_union_grid": ([V, I32, P(U64)], C.c_int),
        "mc_init_multipole": ([V, I32, V, P(D), I32, P(I32), P(I32), P(D), P(D)], C.c_int),
        "mc_lookup_multipole": ([V, SZ, V, V, V, V, P(U64)], C.c_int),
        "mc_lookup_channels": ([V, SZ, V, V, V, V, V], C.c_int),
        "mc_lookup_nuclides": ([V, I32, SZ, V, V, V, V], C.c_int),
        "mc_sort_queue": ([V, SZ, V, V, V, V], C.c_int),
        "mc_hash_bounds": ([P(D), I32, D, D, I32, P(I32)], C.c_int),
        "mc_set_timing": ([V, I32], C.c_int),
        "mc_set_tuning": ([V, P(mc_tuning)], C.c_int),
        "mc_get_tuning": ([V, P(mc_tuning)], C.c_int),
        "mc_autotune": ([V, U64, U64, U64, C.c_char_p, P(mc_tuning)], C.c_int),
        "mc_set_problem_set": ([V, I32, P(mc_problem_desc), I32], C.c_int),
        "mc_run_problem_set": ([V, P(mc_set_opts)], C.c_int),
        "mc_get_problem_tallies": ([V, I32, I32, P(D), P(D), SZ, P(mc_tally_meta)], C.c_int),
        "mc_reset_problem_set": ([V], C.c_int),
        "mc_autotune_problem_set": ([V, C.c_char_p, P(mc_tuning)], C.c_int),
        "mc_mlp_set": ([V, P(C.c_float)], C.c_int),
        "mc_mlp_get": ([V, P(C.c_float)], C.c_int),
        "mc_mlp_forward": ([V, SZ, V, V], C.c_int),
        "mc_mlp_grad": ([V, SZ, V, V, V, P(C.c_float), P(C.c_float)], C.c_int),
        "mc_mlp_train": ([V, SZ, V, V, V, I32, C.c_float, P(C.c_float)], C.c_int),
        "mc_set_weight_windows": ([V, P(mc_ww_desc)], C.c_int),
        "mc_get_importance": ([V, P(D), P(D), P(D), SZ], C.c_int),
        "mc_mlp_init": ([V, U64], C.c_int),
        "mc_importance_samples": ([V, P(D), P(D), P(D), I32, I32, D, D, P(mc_train_opts), V, V, V, P(I32)],
                                  C.c_int),
        "mc_importance_train": ([V, P(mc_train_opts), P(C.c_float), P(I32), P(C.c_float)], C.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _check(ctx, rc):
    if rc != MC_OK:
        msg = load().mc_last_error(ctx).decode() if ctx else ""
        raise MCError(rc, msg)


def _ptr(x):
    """Device pointer of a torch tensor (or an integer / None)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream_handle(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


# ---------------------------------------------------------------------------
# entry points
# ---------------------------------------------------------------------------

def mc_version() -> str:
    return load().mc_version().decode()


def mc_create(device: int = 0, stream=None, allocator="torch"):
    """A context on `device` enqueuing on `stream` (torch's current stream by
    default); allocator "torch": its device memory comes from PyTorch's caching
    allocator, None: from hipMalloc, an mc_alloc instance: from its callbacks
    (the caller keeps it and its callbacks alive while the context lives)."""
    ctx = C.c_void_p()
    if isinstance(allocator, mc_alloc):
        al = C.byref(allocator)
    elif allocator in ("torch", None):
        al = C.byref(_TORCH_ALLOC) if allocator == "torch" else None
    else:
        raise ValueError(f"allocator must be 'torch', None or an mc_alloc, not {allocator!r}")
    rc = load().mc_create(C.byref(ctx), device, _stream_handle(stream), al)
    _check(None, rc)
    return ctx


def mc_destroy(ctx):
    load().mc_destroy(ctx)


def mc_last_error(ctx) -> str:
    return load().mc_last_error(ctx).decode()


def mc_set_stream(ctx, stream=None):
    _check(ctx, load().mc_set_stream(ctx, _stream_handle(stream)))


def mc_init_materials(ctx, E, sig_c, sig_s, awr, mat_nuclides, mat_densities, n_hash_bins=8192):
    """E, sig_c, sig_s: lists of 1-D float64 arrays (one per nuclide); awr: per
    nuclide; mat_nuclides / mat_densities: lists (one per material)."""
    n_nuc = len(E)
    E = [np.ascontiguousarray(e, np.float64) for e in E]
    sc = [np.ascontiguousarray(s, np.float64) for s in sig_c]
    ss = [np.ascontiguousarray(s, np.float64) for s in sig_s]
    grid_len = np.array([e.size for e in E], np.int32)
    PD = C.POINTER(C.c_double)
    pe = (PD * n_nuc)(*[_dp(a) for a in E])
    pc = (PD * n_nuc)(*[_dp(a) for a in sc])
    ps = (PD * n_nuc)(*[_dp(a) for a in ss])
    awr = np.ascontiguousarray(awr, np.float64)
    mat_len = np.array([len(m) for m in mat_nuclides], np.int32)
    mat_nuc = np.ascontiguousarray(np.concatenate([np.asarray(m, np.int32) for m in mat_nuclides]), np.int32)
    mat_dens = np.ascontiguousarray(np.concatenate([np.asarray(d, np.float64) for d in mat_densities]))
    rc = load().mc_init_materials(ctx, n_nuc, _ip(grid_len), pe, pc, ps, _dp(awr), len(mat_len),
                                  _ip(mat_len), _ip(mat_nuc), _dp(mat_dens), int(n_hash_bins))
    _check(ctx, rc)


def mc_init_geometry(ctx, desc: mc_geometry_desc):
    _check(ctx, load().mc_init_geometry(ctx, C.byref(desc)))


def mc_run_batch(ctx, seed: int, first_pid: int, n: int, opts: mc_run_opts | None = None):
    rc = load().mc_run_batch(ctx, seed, first_pid, n, C.byref(opts) if opts is not None else None)
    _check(ctx, rc)


def mc_run_batches(ctx, seed: int, first_pid: int, n: int, n_batches: int, opts: mc_run_opts | None = None):
    rc = load().mc_run_batches(ctx, seed, first_pid, n, n_batches, C.byref(opts) if opts is not None else None)
    _check(ctx, rc)


def mc_get_tallies(ctx, tally_id: int, n_bins: int, raw: bool = False):
    """(mean, stderr, meta); with raw=True also the raw batch sums (S1, S2)."""
    mean = np.zeros(n_bins)
    se = np.zeros(n_bins)
    meta = mc_tally_meta()
    s1 = s2 = None
    if raw:
        s1, s2 = np.zeros(n_bins), np.zeros(n_bins)
        meta.s1, meta.s2 = _dp(s1), _dp(s2)
    _check(ctx, load().mc_get_tallies(ctx, tally_id, _dp(mean), _dp(se), n_bins, C.byref(meta)))
    if raw:
        return mean, se, meta, s1, s2
    return mean, se, meta


def mc_set_tallies(ctx, tally_id: int, s1, s2, n_batches: int, histories: int):
    s1 = np.ascontiguousarray(s1, np.float64)
    s2 = np.ascontiguousarray(s2, np.float64)
    if s1.shape != s2.shape:
        raise ValueError("s1 and s2 differ in size")
    _check(ctx, load().mc_set_tallies(ctx, tally_id, _dp(s1), _dp(s2), s1.size, int(n_batches), int(histories)))


def mc_ww_bootstrap_slope(ctx) -> float:
    a = C.c_double()
    _check(ctx, load().mc_ww_bootstrap_slope(ctx, C.byref(a)))
    return float(a.value)


def mc_reset_tallies(ctx):
    _check(ctx, load().mc_reset_tallies(ctx))


def mc_get_stats(ctx) -> mc_stats:
    s = mc_stats()
    _check(ctx, load().mc_get_stats(ctx, C.byref(s)))
    return s


def mc_lookup_macro(ctx, E, mat, sig_a, sig_s, sorted_: bool = False):
    n = E.numel() if hasattr(E, "numel") else int(E)
    _check(ctx, load().mc_lookup_macro(ctx, n, _ptr(E), _ptr(mat), _ptr(sig_a), _ptr(sig_s),
                                       1 if sorted_ else 0))


MC_NOALLOC_MAX_LOOKUPS = 1 << 20


def mc_lookup_macro_noalloc(ctx, E, mat, sig_a, sig_s, sorted_: bool = False):
    """mc_lookup_macro with the sort's scratch in the library's static device
    array: allocates nothing; at most MC_NOALLOC_MAX_LOOKUPS pairs per call."""
    n = E.numel() if hasattr(E, "numel") else int(E)
    _check(ctx, load().mc_lookup_macro_noalloc(ctx, n, _ptr(E), _ptr(mat), _ptr(sig_a), _ptr(sig_s),
                                               1 if sorted_ else 0))


def mc_init_channels(ctx, channels):
    """Reaction channels: one [grid points, n_chan] float64 array per nuclide
    (None or [] removes them)."""
    if not channels:
        _check(ctx, load().mc_init_channels(ctx, 0, None))
        return
    arrs = [np.ascontiguousarray(c, np.float64) for c in channels]
    k = arrs[0].shape[1]
    if any(a.ndim != 2 or a.shape[1] != k for a in arrs):
        raise ValueError("every nuclide needs a [points, n_chan] array with the same n_chan")
    ptrs = (C.POINTER(C.c_double) * len(arrs))(*[_dp(a) for a in arrs])
    _check(ctx, load().mc_init_channels(ctx, k, ptrs))


class mc_mp_nuclide(C.Structure):
    _fields_ = [("n_poles", C.c_int32), ("n_windows", C.c_int32), ("n_bg", C.c_int32), ("reserved", C.c_int32),
                ("u_lo", C.c_double), ("u_hi", C.c_double),
                ("poles", C.POINTER(C.c_double)), ("res_c", C.POINTER(C.c_double)),
                ("res_s", C.POINTER(C.c_double)), ("win", C.POINTER(C.c_int32)),
                ("bg_c", C.POINTER(C.c_double)), ("bg_s", C.POINTER(C.c_double))]


def mc_init_multipole(ctx, nucs, mat_len, mat_nuc, mat_dens, mat_temp):
    """Multipole nuclides (objects with poles / res_c / res_s complex arrays,
    u_lo, u_hi, win [W, 2], bg_c / bg_s [W, n_bg], awr) and their materials."""
    keep = []

    def arr(a, dt):
        a = np.ascontiguousarray(a, dt)
        keep.append(a)
        return a

    cs = (mc_mp_nuclide * len(nucs))()
    for c, nd in zip(cs, nucs):
        c.n_poles, c.n_windows, c.n_bg = int(np.size(nd.poles)), int(nd.win.shape[0]), int(nd.bg_c.shape[1])
        c.u_lo, c.u_hi = nd.u_lo, nd.u_hi
        c.poles = _dp(arr(np.asarray(nd.poles, np.complex128).view(np.float64), np.float64))
        c.res_c = _dp(arr(np.asarray(nd.res_c, np.complex128).view(np.float64), np.float64))
        c.res_s = _dp(arr(np.asarray(nd.res_s, np.complex128).view(np.float64), np.float64))
        c.win = _ip(arr(nd.win, np.int32))
        c.bg_c = _dp(arr(nd.bg_c, np.float64))
        c.bg_s = _dp(arr(nd.bg_s, np.float64))
    awr = arr([nd.awr for nd in nucs], np.float64)
    ml, mn = arr(mat_len, np.int32), arr(mat_nuc, np.int32)
    md, mt = arr(mat_dens, np.float64), arr(mat_temp, np.float64)
    _check(ctx, load().mc_init_multipole(ctx, len(nucs), C.cast(cs, C.c_void_p), _dp(awr), ml.size, _ip(ml), _ip(mn),
                                         _dp(md), _dp(mt)))


def mc_lookup_multipole(ctx, E, mat, sig_a, sig_s, count_poles: bool = False):
    n = E.numel()
    cnt = C.c_uint64(0)
    _check(ctx, load().mc_lookup_multipole(ctx, n, _ptr(E), _ptr(mat), _ptr(sig_a), _ptr(sig_s),
                                           C.byref(cnt) if count_poles else None))
    return int(cnt.value) if count_poles else None


def mc_set_union_grid(ctx, on: bool = True) -> int:
    """Unionized-grid lookups on (device bytes of the tables) or off."""
    b = C.c_uint64(0)
    _check(ctx, load().mc_set_union_grid(ctx, 1 if on else 0, C.byref(b)))
    return int(b.value)


def mc_lookup_channels(ctx, E, mat, out, sig_a=None, sig_s=None):
    n = E.numel() if hasattr(E, "numel") else int(E)
    _check(ctx, load().mc_lookup_channels(ctx, n, _ptr(E), _ptr(mat), _ptr(out), _ptr(sig_a), _ptr(sig_s)))


def mc_lookup_nuclides(ctx, mat: int, E, idx=None, sig_c=None, sig_s=None):
    _check(ctx, load().mc_lookup_nuclides(ctx, mat, E.numel(), _ptr(E), _ptr(idx), _ptr(sig_c),
                                          _ptr(sig_s)))


def mc_sort_queue(ctx, E, mat, perm, keys_sorted=None):
    _check(ctx, load().mc_sort_queue(ctx, E.numel(), _ptr(E), _ptr(mat), _ptr(perm),
                                     _ptr(keys_sorted)))


def mc_set_tuning(ctx, **fields):
    """Fields of mc_tuning by name (missing ones: 0 = library default)."""
    t = mc_tuning()
    for k, v in fields.items():
        if k not in mc_tuning.KEYS:
            raise KeyError(k)
        setattr(t, k, int(v))
    _check(ctx, load().mc_set_tuning(ctx, C.byref(t)))


def mc_autotune(ctx, seed: int, first_pid: int, n: int, cache_path: str | None = None) -> dict:
    t = mc_tuning()
    _check(ctx, load().mc_autotune(ctx, seed, first_pid, n, cache_path.encode() if cache_path else None,
                                   C.byref(t)))
    return t.as_dict()


def mc_set_problem_set(ctx, problems, n_hash_bins: int = 8192):
    """problems: list of dicts with keys E, sig_c, sig_s, awr, mat_nuclides,
    mat_densities (as mc_init_materials), geometry (an mc_geometry_desc),
    histories, seed, first_pid."""
    keep = []
    arr = (mc_problem_desc * len(problems))()
    PD = C.POINTER(C.c_double)
    for i, p in enumerate(problems):
        E = [np.ascontiguousarray(e, np.float64) for e in p["E"]]
        sc = [np.ascontiguousarray(s, np.float64) for s in p["sig_c"]]
        ss = [np.ascontiguousarray(s, np.float64) for s in p["sig_s"]]
        n = len(E)
        grid_len = np.array([e.size for e in E], np.int32)
        pe = (PD * n)(*[_dp(x) for x in E])
        pc = (PD * n)(*[_dp(x) for x in sc])
        ps = (PD * n)(*[_dp(x) for x in ss])
        awr = np.ascontiguousarray(p["awr"], np.float64)
        mat_len = np.array([len(m) for m in p["mat_nuclides"]], np.int32)
        mat_nuc = np.ascontiguousarray(np.concatenate([np.asarray(m, np.int32) for m in p["mat_nuclides"]]), np.int32)
        mat_dens = np.ascontiguousarray(np.concatenate([np.asarray(d, np.float64) for d in p["mat_densities"]]))
        keep += [E, sc, ss, grid_len, pe, pc, ps, awr, mat_len, mat_nuc, mat_dens, p["geometry"]]
        d = arr[i]
        d.n_nuc = n
        d.grid_len = _ip(grid_len)
        d.E, d.sig_c, d.sig_s = pe, pc, ps
        d.awr = _dp(awr)
        d.n_mat = len(mat_len)
        d.mat_len, d.mat_nuc, d.mat_dens = _ip(mat_len), _ip(mat_nuc), _dp(mat_dens)
        d.geometry = C.pointer(p["geometry"])
        d.histories, d.seed, d.first_pid = int(p["histories"]), int(p["seed"]), int(p["first_pid"])
    _check(ctx, load().mc_set_problem_set(ctx, len(problems), arr, int(n_hash_bins)))
    del keep


def mc_run_problem_set(ctx, use_graph: bool = False, max_events: int = 0, history_log=None):
    o = mc_set_opts()
    o.use_graph = 1 if use_graph else 0
    o.max_events = int(max_events)
    o.history_log = _ptr(history_log)
    _check(ctx, load().mc_run_problem_set(ctx, C.byref(o)))


def mc_get_problem_tallies(ctx, problem: int, tally_id: int, n_bins: int):
    mean = np.zeros(n_bins)
    se = np.zeros(n_bins)
    meta = mc_tally_meta()
    _check(ctx, load().mc_get_problem_tallies(ctx, problem, tally_id, _dp(mean), _dp(se), n_bins, C.byref(meta)))
    return mean, se, meta


def mc_reset_problem_set(ctx):
    _check(ctx, load().mc_reset_problem_set(ctx))


def mc_autotune_problem_set(ctx, cache_path: str | None = None) -> dict:
    t = mc_tuning()
    _check(ctx, load().mc_autotune_problem_set(ctx, cache_path.encode() if cache_path else None, C.byref(t)))
    return t.as_dict()


MC_MLP_NPAR = 4545


def _fp(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def mc_mlp_set(ctx, params):
    """Load the flat parameter vector (MC_MLP_NPAR values) and reset Adam."""
    p = np.ascontiguousarray(params, np.float32)
    if p.size != MC_MLP_NPAR:
        raise ValueError(f"mc_mlp_set: {p.size} parameters, expected {MC_MLP_NPAR}")
    _check(ctx, load().mc_mlp_set(ctx, _fp(p)))


def mc_mlp_get(ctx) -> np.ndarray:
    p = np.zeros(MC_MLP_NPAR, np.float32)
    _check(ctx, load().mc_mlp_get(ctx, _fp(p)))
    return p


def mc_mlp_forward(ctx, n: int, features, out):
    """features: device float32 [n, 4]; out: device float32 [n]."""
    _check(ctx, load().mc_mlp_forward(ctx, int(n), _ptr(features), _ptr(out)))


def mc_mlp_grad(ctx, n: int, features, target, weight):
    """Returns (gradient [MC_MLP_NPAR] float32, loss)."""
    g = np.zeros(MC_MLP_NPAR, np.float32)
    loss = C.c_float()
    _check(ctx, load().mc_mlp_grad(ctx, int(n), _ptr(features), _ptr(target), _ptr(weight), _fp(g),
                                   C.byref(loss)))
    return g, float(loss.value)


def mc_mlp_train(ctx, n: int, features, target, weight, steps: int, lr: float) -> np.ndarray:
    """Returns the loss before each of the `steps` Adam steps."""
    curve = np.zeros(int(steps), np.float32)
    _check(ctx, load().mc_mlp_train(ctx, int(n), _ptr(features), _ptr(target), _ptr(weight), int(steps),
                                    float(lr), _fp(curve)))
    return curve


def mc_set_weight_windows(ctx, kind=MC_WW_OFF, lin=(0.0, 0.0, 0.0), length=200.0, kappa=3.0, ratio=5.0,
                          n_max=10, depth=24, imp_nx=0, imp_ne=0, imp_x0=0.0, imp_x1=200.0, ln_lo=0.0, ln_hi=0.0):
    d = mc_ww_desc()
    d.kind, d.n_max, d.depth = int(kind), int(n_max), int(depth)
    d.imp_nx, d.imp_ne = int(imp_nx), int(imp_ne)
    d.lin = (C.c_double * 3)(*[float(v) for v in lin])
    d.length, d.kappa, d.ratio = float(length), float(kappa), float(ratio)
    d.imp_x0, d.imp_x1 = float(imp_x0), float(imp_x1)
    d.ln_lo, d.ln_hi = float(ln_lo), float(ln_hi)
    _check(ctx, load().mc_set_weight_windows(ctx, C.byref(d)))


def mc_get_importance(ctx, n_cells: int):
    """Returns (num, den, cnt), each [n_cells] float64."""
    num, den, cnt = np.zeros(n_cells), np.zeros(n_cells), np.zeros(n_cells)
    _check(ctx, load().mc_get_importance(ctx, _dp(num), _dp(den), _dp(cnt), int(n_cells)))
    return num, den, cnt


def train_opts(steps=2000, replicas=4, lr=1e-2, min_credits=10.0, rel_floor=0.1, length=200.0, seed=0):
    o = mc_train_opts()
    o.steps, o.replicas, o.lr = int(steps), int(replicas), float(lr)
    o.min_credits, o.rel_floor, o.length, o.seed = float(min_credits), float(rel_floor), float(length), int(seed)
    return o


def mc_mlp_init(ctx, seed: int = 0):
    _check(ctx, load().mc_mlp_init(ctx, int(seed)))


def mc_importance_samples(ctx, num, den, cnt, nx: int, ne: int, x0: float, x1: float, opts, features, target,
                          weight) -> int:
    """Host sums in, device samples out (features [cells * replicas, 4] float32 ...); returns the count."""
    num = np.ascontiguousarray(num, np.float64)
    den = np.ascontiguousarray(den, np.float64)
    cnt = np.ascontiguousarray(cnt, np.float64)
    n = C.c_int32()
    _check(ctx, load().mc_importance_samples(ctx, _dp(num), _dp(den), _dp(cnt), int(nx), int(ne), float(x0),
                                             float(x1), C.byref(opts), _ptr(features), _ptr(target), _ptr(weight),
                                             C.byref(n)))
    return int(n.value)


def mc_importance_train(ctx, opts):
    """Returns (loss curve [steps] float32, number of samples, (smallest, largest target))."""
    curve = np.zeros(max(int(opts.steps), 1), np.float32)
    n = C.c_int32()
    rng = np.zeros(2, np.float32)
    _check(ctx, load().mc_importance_train(ctx, C.byref(opts), _fp(curve), C.byref(n), _fp(rng)))
    return curve, int(n.value), (float(rng[0]), float(rng[1]))


def mc_get_tuning(ctx) -> dict:
    t = mc_tuning()
    _check(ctx, load().mc_get_tuning(ctx, C.byref(t)))
    return t.as_dict()


def mc_set_timing(ctx, on: bool):
    _check(ctx, load().mc_set_timing(ctx, 1 if on else 0))


def mc_hash_bounds(E, emin: float, emax: float, M: int) -> np.ndarray:
    E = np.ascontiguousarray(E, np.float64)
    lo = np.zeros(M + 1, np.int32)
    rc = load().mc_hash_bounds(_dp(E), E.size, emin, emax, M, _ip(lo))
    _check(None, rc)
    return lo
