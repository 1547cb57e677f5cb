"""Marshalling of a problem description (an object with the attributes of
``mcsynth.Problem``: nuclides, materials, geometry, source, tally,
energy_cutoff, n_hash_bins) into the C ABI, and a small context wrapper.

Nothing here computes any part of the transport path; it only fills the
library's structs and forwards calls.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import mc


def geometry_desc(prob):
    """Fill an mc_geometry_desc; returns (desc, keep-alive arrays)."""
    g, s, t = prob.geometry, prob.source, prob.tally
    keep = []

    def arr(a, dt):
        a = np.ascontiguousarray(a, dt)
        keep.append(a)
        return a

    d = mc.mc_geometry_desc()
    d.kind, d.material = g.kind, g.material
    d.nx, d.ny, d.pitch, d.radius, d.z0, d.z1 = g.nx, g.ny, g.pitch, g.radius, g.z0, g.z1
    if g.pin_material is not None:
        d.pin_material = arr(g.pin_material, np.int32).ctypes.data_as(C.POINTER(C.c_int32))
    d.moderator_material = g.moderator_material
    d.bc = (C.c_int32 * 6)(*g.bc)
    if g.x_edges is not None:
        d.n_layers = len(g.x_edges) - 1
        d.x_edges = arr(g.x_edges, np.float64).ctypes.data_as(C.POINTER(C.c_double))
        d.layer_material = arr(g.layer_material, np.int32).ctypes.data_as(C.POINTER(C.c_int32))
    d.source_kind = s.kind
    d.source_pos = (C.c_double * 3)(*s.position)
    d.source_box = (C.c_double * 6)(*s.box)
    d.source_dir = (C.c_double * 3)(*s.direction)
    d.source_energy = s.energy
    d.tally_kind = t.kind
    if t.energy_edges is not None:
        d.n_energy_bins = len(t.energy_edges) - 1
        d.energy_edges = arr(t.energy_edges, np.float64).ctypes.data_as(C.POINTER(C.c_double))
    d.mesh_dims = (C.c_int32 * 3)(*t.mesh_dims)
    d.mesh_box = (C.c_double * 6)(*t.mesh_box)
    d.energy_cutoff = prob.energy_cutoff
    return d, keep


def run_opts(in_flight=0, sort_min=0, no_tally=False, time_kernels=False, max_events=0, max_lost=0,
             history_log=None):
    o = mc.mc_run_opts()
    o.in_flight = int(in_flight)
    o.sort_min = int(sort_min)
    o.no_tally = 1 if no_tally else 0
    o.time_kernels = 1 if time_kernels else 0
    o.max_events = int(max_events)
    o.max_lost = int(max_lost)
    o.history_log = mc._ptr(history_log)
    return o


class Transport:
    """One library context holding one problem."""

    def __init__(self, prob, device: int = 0, stream=None, allocator: str | None = "torch"):
        self.prob = prob
        self.ctx = mc.mc_create(device, stream, allocator)
        try:
            mc.mc_init_materials(self.ctx, [n.E for n in prob.nuclides], [n.sig_c for n in prob.nuclides],
                                 [n.sig_s for n in prob.nuclides], [n.awr for n in prob.nuclides],
                                 [m.nuclides for m in prob.materials], [m.densities for m in prob.materials],
                                 prob.n_hash_bins)
            desc, keep = geometry_desc(prob)
            mc.mc_init_geometry(self.ctx, desc)
            del keep
            self.set_weight_windows(getattr(prob, "ww", None), getattr(prob, "imp", None))
            chans = getattr(prob, "channels", None)
            if chans:
                mc.mc_init_channels(self.ctx, chans)
        except Exception:
            mc.mc_destroy(self.ctx)
            raise
        self.n_bins = prob.n_bins
        self.n_reaction = len(prob.materials) * (chans[0].shape[1] if chans else 0)

    def set_weight_windows(self, ww=None, imp=None):
        """Weight windows (an object with the attributes of mcsynth.WeightWindows)
        and the importance grid (mcsynth.ImportanceGrid); the network of an
        MLP window is loaded into the context first."""
        kind = ww.kind if ww is not None else mc.MC_WW_OFF
        if kind == mc.MC_WW_MLP:
            mc.mc_mlp_set(self.ctx, ww.mlp)
        kw = {}
        if ww is not None:
            kw.update(kind=kind, lin=ww.lin, length=ww.length, kappa=ww.kappa, ratio=ww.ratio, n_max=ww.n_max,
                      depth=ww.depth, ln_lo=getattr(ww, "ln_lo", 0.0), ln_hi=getattr(ww, "ln_hi", 0.0))
        if imp is not None and imp.nx > 0:
            kw.update(imp_nx=imp.nx, imp_ne=imp.ne, imp_x0=imp.x0, imp_x1=imp.x1)
        mc.mc_set_weight_windows(self.ctx, **kw)
        self.n_imp_cells = imp.nx * imp.ne if imp is not None else 0

    def importance(self):
        """(num, den, cnt) of the importance grid, [3, cells]."""
        return np.stack(mc.mc_get_importance(self.ctx, self.n_imp_cells))

    def run_batch(self, seed, first_pid, n, **opts):
        mc.mc_run_batch(self.ctx, seed, first_pid, n, run_opts(**opts))

    def run_batches(self, seed, first_pid, n, n_batches, **opts):
        mc.mc_run_batches(self.ctx, seed, first_pid, n, n_batches, run_opts(**opts))

    def _bins(self, tally_id):
        return {mc.MC_T_GLOBAL: mc.MC_N_GLOBAL, mc.MC_T_REACTION: self.n_reaction}.get(tally_id, self.n_bins)

    def tallies(self, tally_id):
        mean, se, meta = mc.mc_get_tallies(self.ctx, tally_id, self._bins(tally_id))
        return mean, se, meta

    def checkpoint(self) -> dict:
        """Raw batch sums of every tally, the batch count and history total:
        what restore() needs to resume between batches."""
        ids = [mc.MC_T_FLUX_TRACK, mc.MC_T_FLUX_COLLISION, mc.MC_T_GLOBAL]
        if self.n_reaction:
            ids.append(mc.MC_T_REACTION)
        out = {"tallies": {}}
        for k in ids:
            _, _, meta, s1, s2 = mc.mc_get_tallies(self.ctx, k, self._bins(k), raw=True)
            out["tallies"][k] = (s1, s2)
            out["n_batches"], out["histories"] = int(meta.n_batches), int(meta.histories)
        return out

    def restore(self, state: dict):
        for k, (s1, s2) in state["tallies"].items():
            mc.mc_set_tallies(self.ctx, k, s1, s2, state["n_batches"], state["histories"])

    def reset(self):
        mc.mc_reset_tallies(self.ctx)

    def stats(self) -> dict:
        return mc.mc_get_stats(self.ctx).as_dict()

    def close(self):
        if self.ctx is not None:
            mc.mc_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def problem_entry(prob, first_pid: int = 0):
    """One problem of a problem set (dict for mc.mc_set_problem_set) plus the
    arrays its geometry description points at."""
    desc, keep = geometry_desc(prob)
    return {"E": [n.E for n in prob.nuclides], "sig_c": [n.sig_c for n in prob.nuclides],
            "sig_s": [n.sig_s for n in prob.nuclides], "awr": [n.awr for n in prob.nuclides],
            "mat_nuclides": [m.nuclides for m in prob.materials],
            "mat_densities": [m.densities for m in prob.materials],
            "geometry": desc, "histories": prob.histories, "seed": prob.seed, "first_pid": first_pid,
            "_keep": keep}


class ProblemSet:
    """One library context holding a problem set."""

    def __init__(self, probs, device: int = 0, stream=None, n_hash_bins: int = 8192):
        self.probs = probs
        self.ctx = mc.mc_create(device, stream)
        try:
            entries = [problem_entry(p) for p in probs]
            mc.mc_set_problem_set(self.ctx, entries, n_hash_bins)
            del entries
        except Exception:
            mc.mc_destroy(self.ctx)
            raise

    def run_batch(self, use_graph=False, max_events=0, history_log=None):
        mc.mc_run_problem_set(self.ctx, use_graph, max_events, history_log)

    def tallies(self, problem, tally_id):
        nb = mc.MC_N_GLOBAL if tally_id == mc.MC_T_GLOBAL else self.probs[problem].n_bins
        return mc.mc_get_problem_tallies(self.ctx, problem, tally_id, nb)

    def reset(self):
        mc.mc_reset_problem_set(self.ctx)

    def stats(self) -> dict:
        return mc.mc_get_stats(self.ctx).as_dict()

    def close(self):
        if self.ctx is not None:
            mc.mc_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
