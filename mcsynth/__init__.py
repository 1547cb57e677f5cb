"""Seeded synthetic inputs for the transport problems.

This module is shared by the CPU oracle wrapper and by the GPU library's
callers.  It draws nuclide data, material compositions and problem
descriptions from ``numpy.random.default_rng(data_seed)`` and holds none of the
transport method's arithmetic: no grid search, no interpolation, no macroscopic
sums, no tracking.  The transport random numbers (Philox) are *not* drawn here;
each side implements that generator itself.

The paper's real nuclear data and its reactor problems are not available, so
every nuclide is synthetic: on its energy grid E_j the tabulated capture and
elastic-scattering cross sections are

    sigma_x(E) = a_x + b_x * sqrt(E_th / E)
                 + sum_{r=1..10} h_{x,r} / (1 + ((E - E_r) / (Gamma_r / 2))**2)

(a constant, a 1/v term and ten Lorentzian resonances; x in {c, s}), and the
tabulated values are the data: the physics "truth" between grid points is their
linear interpolation, as in a continuous-energy library.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

EMIN = 1.0e-5        # eV, lower end of every energy grid and the energy cutoff
EMAX = 2.0e7         # eV, upper end of every energy grid
E_THERMAL = 0.0253   # eV, reference energy of the 1/v term
SOURCE_ENERGY = 2.0e6  # eV

# geometry / boundary / source / tally kinds (plain integers, mirrored by each side)
GEOM_INFINITE, GEOM_LATTICE, GEOM_SLAB = 0, 1, 2
BC_REFLECT, BC_VACUUM = 0, 1
SRC_POINT, SRC_BOX, SRC_BEAM = 0, 1, 2
TALLY_ENERGY, TALLY_PIN, TALLY_MESH, TALLY_SLAB = 0, 1, 2, 3


@dataclass
class Nuclide:
    E: np.ndarray        # float64, strictly increasing, eV
    sig_c: np.ndarray    # float64 capture cross section, barns
    sig_s: np.ndarray    # float64 elastic cross section, barns
    awr: float           # target mass in neutron masses (A)


@dataclass
class Material:
    nuclides: np.ndarray   # int32 nuclide ids, in material order
    densities: np.ndarray  # float64 atom densities, atoms/(barn cm)


@dataclass
class Geometry:
    kind: int = GEOM_INFINITE
    material: int = 0                     # infinite medium
    nx: int = 0                           # lattice cells along x / y
    ny: int = 0
    pitch: float = 0.0
    radius: float = 0.0
    z0: float = 0.0
    z1: float = 0.0
    pin_material: Optional[np.ndarray] = None   # int32 [ny*nx], -1 = no cylinder
    moderator_material: int = 0
    bc: tuple = (BC_REFLECT,) * 6         # x-, x+, y-, y+, z-, z+
    x_edges: Optional[np.ndarray] = None  # slab layer edges along x
    layer_material: Optional[np.ndarray] = None


@dataclass
class Source:
    kind: int = SRC_POINT
    position: tuple = (0.0, 0.0, 0.0)
    box: tuple = (0.0, 0.0, 0.0, 0.0, 0.0, 0.0)  # x0, x1, y0, y1, z0, z1
    direction: tuple = (1.0, 0.0, 0.0)
    energy: float = SOURCE_ENERGY


@dataclass
class Tally:
    kind: int = TALLY_ENERGY
    energy_edges: Optional[np.ndarray] = None  # float64, n_bins + 1
    mesh_dims: tuple = (1, 1, 1)
    mesh_box: tuple = (0.0, 1.0, 0.0, 1.0, 0.0, 1.0)

    def n_bins(self, geom: Geometry) -> int:
        if self.kind == TALLY_ENERGY:
            return len(self.energy_edges) - 1
        if self.kind == TALLY_PIN:
            return geom.nx * geom.ny
        if self.kind == TALLY_MESH:
            return int(np.prod(self.mesh_dims))
        if self.kind == TALLY_SLAB:
            return len(geom.x_edges) - 1
        raise ValueError(self.kind)


WW_OFF, WW_LINEAR, WW_MLP = 0, 1, 2


@dataclass
class WeightWindows:
    """Weight windows from an importance map ln I(x, y, z, E): linear in the
    features (``lin`` = c0, c1, c2 for c0 + c1 x/L + c2 (ln E - ln 1e-5)/ln(2e12))
    or the importance network (``mlp``: its 4545 parameters, W1[4][64], b1,
    W2[64][64], b2, w3[64], b3 in that order, row-major).  Window at a point:
    w_L = exp(ln I_src - ln I) / kappa, w_U = ratio w_L; ln I is clamped to
    [ln_lo, ln_hi] when ln_lo < ln_hi."""
    kind: int = WW_OFF
    lin: tuple = (0.0, 0.0, 0.0)
    mlp: Optional[np.ndarray] = None
    length: float = 200.0
    kappa: float = 3.0
    ratio: float = 5.0
    n_max: int = 10
    depth: int = 24
    ln_lo: float = 0.0
    ln_hi: float = 0.0


@dataclass
class ImportanceGrid:
    """x by ln E grid of the forward importance estimate (nx = 0: off)."""
    nx: int = 0
    ne: int = 0
    x0: float = 0.0
    x1: float = 200.0

    @property
    def cells(self) -> int:
        return self.nx * self.ne


@dataclass
class Problem:
    name: str
    nuclides: List[Nuclide]
    materials: List[Material]
    geometry: Geometry
    source: Source
    tally: Tally
    energy_cutoff: float = EMIN
    n_hash_bins: int = 8192
    histories: int = 10_000
    batches: int = 10
    seed: int = 1                # transport (Philox key) seed
    ww: WeightWindows = field(default_factory=WeightWindows)
    imp: ImportanceGrid = field(default_factory=ImportanceGrid)
    meta: dict = field(default_factory=dict)
    # reaction channels: per nuclide a [grid points, n_chan] float64 array (or None)
    channels: Optional[List[np.ndarray]] = None

    @property
    def n_bins(self) -> int:
        return self.tally.n_bins(self.geometry)

    @property
    def n_chan(self) -> int:
        return 0 if not self.channels else int(self.channels[0].shape[1])

    def data_bytes(self) -> int:
        b = sum(n.E.nbytes + n.sig_c.nbytes + n.sig_s.nbytes for n in self.nuclides)
        return int(b + (sum(c.nbytes for c in self.channels) if self.channels else 0))


# ---------------------------------------------------------------------------
# nuclide data
# ---------------------------------------------------------------------------

def _log_uniform(rng, lo, hi, size=None):
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size))


def log_uniform_grid(n: int) -> np.ndarray:
    """n points uniform in ln E over [EMIN, EMAX] with both ends set exactly."""
    g = np.exp(np.linspace(np.log(EMIN), np.log(EMAX), n))
    g[0], g[-1] = EMIN, EMAX
    return g


# offsets (in widths) of the points clustered around each resonance
_CLUSTER_T = np.array([0.0, 0.05, 0.1, 0.2, 0.3, 0.4, 0.5, 0.65, 0.8, 1.0, 1.25, 1.5, 2.0,
                       2.5, 3.0, 4.0, 5.0, 7.0, 10.0, 15.0, 25.0, 40.0])
_CLUSTER_T = np.concatenate([-_CLUSTER_T[:0:-1], _CLUSTER_T])


def clustered_grid(n_target: int, e_res: np.ndarray, g_res: np.ndarray) -> np.ndarray:
    """Log-uniform base grid unioned with points clustered at E_r + Gamma_r * t."""
    pts = (e_res[:, None] + g_res[:, None] * _CLUSTER_T[None, :]).ravel()
    pts = pts[(pts > EMIN) & (pts < EMAX)]
    n_base = max(16, n_target - pts.size)
    g = np.unique(np.concatenate([log_uniform_grid(n_base), pts]))
    assert g[0] == EMIN and g[-1] == EMAX
    return g


def _resonance_params(rng, n_res=10):
    e_res = _log_uniform(rng, 1.0, 1.0e5, n_res)
    g_res = e_res * 10.0 ** rng.uniform(-3.0, -1.5, n_res)
    return e_res, g_res


def _channel(E, a, b, e_res, g_res, h):
    s = a + b * np.sqrt(E_THERMAL / E)
    for er, gr, hr in zip(e_res, g_res, h):
        s = s + hr / (1.0 + ((E - er) / (0.5 * gr)) ** 2)
    return s


def make_nuclide(rng, awr: float, n_points: int, grid: str = "loguniform",
                 n_res: int = 10, literal_scatter: bool = False) -> Nuclide:
    """Draw one synthetic nuclide (see module docstring for the formula).

    a_c = 0; a_s ~ U[2, 20] b (potential scattering; ``literal_scatter`` sets it to 0);
    b_c ~ logU[0.1, 100] b; b_s ~ logU[0.01, 1] b; resonance energies E_r ~ logU[1, 1e5] eV,
    widths Gamma_r = E_r * 10**U[-3, -1.5], heights h ~ logU[10, 1e4] b, the resonance
    positions shared by both channels and the heights drawn per channel.
    """
    e_res, g_res = _resonance_params(rng, n_res)
    if grid == "loguniform":
        E = log_uniform_grid(n_points)
    elif grid == "clustered":
        E = clustered_grid(n_points, e_res, g_res)
    else:
        raise ValueError(grid)
    a_s = 0.0 if literal_scatter else rng.uniform(2.0, 20.0)
    b_c = _log_uniform(rng, 0.1, 100.0)
    b_s = _log_uniform(rng, 0.01, 1.0)
    h_c = _log_uniform(rng, 10.0, 1.0e4, n_res)
    h_s = _log_uniform(rng, 10.0, 1.0e4, n_res)
    sc = _channel(E, 0.0, b_c, e_res, g_res, h_c)
    ss = _channel(E, a_s, b_s, e_res, g_res, h_s)
    assert np.all(np.diff(E) > 0) and np.all(sc >= 0) and np.all(ss >= 0)
    return Nuclide(E=E.astype(np.float64), sig_c=sc.astype(np.float64),
                   sig_s=ss.astype(np.float64), awr=float(awr))


def make_channels(rng, nuc: Nuclide, n_chan: int, n_res: int = 3) -> np.ndarray:
    """[grid points, n_chan] reaction-channel cross sections on the nuclide's
    grid: per channel a constant a ~ U[0, 2] b, a 1/v term b ~ logU[0.01, 10] b
    and n_res Lorentzians (energies and widths drawn like the nuclide's,
    heights logU[1, 1e3] b)."""
    out = np.empty((nuc.E.size, n_chan))
    for x in range(n_chan):
        e_res, g_res = _resonance_params(rng, n_res)
        a = rng.uniform(0.0, 2.0)
        b = _log_uniform(rng, 0.01, 10.0)
        h = _log_uniform(rng, 1.0, 1.0e3, n_res)
        out[:, x] = _channel(nuc.E, a, b, e_res, g_res, h)
    assert np.all(out >= 0)
    return np.ascontiguousarray(out, np.float64)


def with_channels(prob: "Problem", n_chan: int, data_seed: int = 9009) -> "Problem":
    """The problem with n_chan synthetic reaction channels on every nuclide
    (the per-nuclide reaction data a depletion tally gathers)."""
    rng = np.random.default_rng(data_seed)
    prob.channels = [make_channels(rng, n, n_chan) for n in prob.nuclides]
    return prob


@dataclass
class MultipoleNuclide:
    """Windowed-multipole data of one nuclide (u = sqrt(E)): poles (Im < 0),
    capture and scattering residues, [n_windows, 2] pole ranges of the even
    windows over [u_lo, u_hi], and per window background coefficients of
    u^-1, u^0, u^1."""
    poles: np.ndarray   # complex128 [P], sorted by real part
    res_c: np.ndarray   # complex128 [P]
    res_s: np.ndarray   # complex128 [P]
    u_lo: float
    u_hi: float
    win: np.ndarray     # int32 [W, 2]
    bg_c: np.ndarray    # float64 [W, 3]
    bg_s: np.ndarray    # float64 [W, 3]
    awr: float


def make_multipole_nuclide(rng, awr: float, n_res: int = 20, n_windows: int = 1024,
                           reach: float = 2.0) -> MultipoleNuclide:
    """Synthetic multipole nuclide: resonances E_r ~ logU[1, 1e5] eV with
    widths Gamma = E_r 10^U[-3, -1.5] become poles sqrt(E_r) - i Gamma / (4
    sqrt(E_r)); a residue h gamma E_r gives a resonance of peak h barns (capture
    heights logU[10, 1e4] b with real residues, scattering heights logU[10, 1e3] b
    with a phase of up to 0.2 rad); background 1/v capture b_c sqrt(0.0253 / E)
    and constant potential scattering a_s.  Window w holds the poles within
    reach + 1/2 window widths of its centre."""
    e_r = np.sort(_log_uniform(rng, 1.0, 1.0e5, n_res))
    gam_e = e_r * 10.0 ** rng.uniform(-3.0, -1.5, n_res)
    a = np.sqrt(e_r)
    g = gam_e / (4.0 * a)
    poles = a - 1j * g
    h_c = _log_uniform(rng, 10.0, 1.0e4, n_res)
    h_s = _log_uniform(rng, 10.0, 1.0e3, n_res)
    res_c = (h_c * g * e_r).astype(np.complex128)
    res_s = h_s * g * e_r * np.exp(1j * rng.uniform(-0.2, 0.2, n_res))
    u_lo, u_hi = np.sqrt(EMIN), np.sqrt(EMAX)
    du = (u_hi - u_lo) / n_windows
    centre = u_lo + (np.arange(n_windows) + 0.5) * du
    lo = np.searchsorted(a, centre - (reach + 0.5) * du, side="left")
    hi = np.searchsorted(a, centre + (reach + 0.5) * du, side="right")
    win = np.stack([lo, hi], 1).astype(np.int32)
    b_c = _log_uniform(rng, 0.1, 100.0) * np.sqrt(E_THERMAL)
    a_s = rng.uniform(2.0, 20.0)
    bg_c = np.tile([b_c, 0.0, 0.0], (n_windows, 1))
    bg_s = np.tile([0.0, a_s, 0.0], (n_windows, 1))
    return MultipoleNuclide(poles=poles, res_c=res_c, res_s=res_s, u_lo=float(u_lo), u_hi=float(u_hi), win=win,
                            bg_c=bg_c, bg_s=bg_s, awr=float(awr))


def multipole_material(n_nuclides: int = 300, data_seed: int = 7007, n_res: int = 200):
    """n_nuclides synthetic multipole nuclides of n_res resonances each (A = 1
    first, then U[2, 240]) and densities log-uniform in [1e-6, 1e-2]
    atoms/(b cm)."""
    rng = np.random.default_rng(data_seed)
    awr = np.concatenate([[1.0], rng.uniform(2.0, 240.0, n_nuclides - 1)])
    nucs = [make_multipole_nuclide(rng, a, n_res=n_res) for a in awr]
    dens = _log_uniform(rng, 1e-6, 1e-2, n_nuclides)
    return nucs, np.arange(n_nuclides, dtype=np.int32), dens


def constant_nuclide(sig_c: float, sig_s: float, awr: float, n_points: int = 2000) -> Nuclide:
    """A nuclide whose tabulated cross sections are constant (closed-form tests)."""
    E = log_uniform_grid(n_points)
    return Nuclide(E=E, sig_c=np.full_like(E, sig_c), sig_s=np.full_like(E, sig_s), awr=float(awr))


def _analytic_sigma_t(nuc: Nuclide, E: float) -> float:
    # only used to scale densities: the nearest tabulated point, no interpolation
    j = int(np.argmin(np.abs(nuc.E - E)))
    return float(nuc.sig_c[j] + nuc.sig_s[j])


def make_material(rng, nuclides: List[Nuclide], ids, target_sigma_t: float,
                  density_range=(1.0e-6, 1.0e-2), fixed_fraction=None) -> Material:
    """Densities ~ logU[density_range], rescaled so Sigma_t(2 MeV) ~= target_sigma_t (1/cm).

    ``fixed_fraction`` = (position, fraction) forces the nuclide at that position of ``ids``
    to carry the given fraction of Sigma_t(2 MeV) (a moderator's hydrogen-like nuclide).
    """
    ids = np.asarray(ids, dtype=np.int32)
    dens = _log_uniform(rng, density_range[0], density_range[1], ids.size)
    st = np.array([_analytic_sigma_t(nuclides[k], SOURCE_ENERGY) for k in ids])
    if fixed_fraction is not None:
        pos, frac = fixed_fraction
        others = np.delete(np.arange(ids.size), pos)
        rest = float(np.sum(dens[others] * st[others]))
        dens[others] *= (1.0 - frac) * target_sigma_t / rest
        dens[pos] = frac * target_sigma_t / st[pos]
    else:
        dens *= target_sigma_t / float(np.sum(dens * st))
    return Material(nuclides=ids, densities=dens.astype(np.float64))


def energy_edges(n_bins: int) -> np.ndarray:
    return log_uniform_grid(n_bins + 1)


# ---------------------------------------------------------------------------
# problems
# ---------------------------------------------------------------------------

def c1_problem(data_seed: int = 1001, seed: int = 1, histories: int = 10_000,
               batches: int = 10) -> Problem:
    """Infinite homogeneous medium: one material of 4 nuclides (A = 1, 12, 56, 238), each on a
    2,000-point log-uniform grid over [1e-5 eV, 20 MeV]; isotropic 2 MeV point source at the
    origin; 50-bin log-energy track-length flux tally."""
    rng = np.random.default_rng(data_seed)
    awrs = [1.0, 12.0, 56.0, 238.0]
    nucs = [make_nuclide(rng, a, 2000, "loguniform") for a in awrs]
    mat = make_material(rng, nucs, [0, 1, 2, 3], 0.5, fixed_fraction=(0, 0.5))
    return Problem(name="c1_infinite_4nuc", nuclides=nucs, materials=[mat],
                   geometry=Geometry(kind=GEOM_INFINITE, material=0),
                   source=Source(kind=SRC_POINT), tally=Tally(TALLY_ENERGY, energy_edges(50)),
                   histories=histories, batches=batches, seed=seed)


def infinite_many_nuclides_problem(n_nuclides: int = 60, data_seed: int = 1101, seed: int = 7,
                                   histories: int = 4000, n_points: int = 2000) -> Problem:
    """Infinite medium of one material of many synthetic nuclides (the first
    hydrogen-like at half of Sigma_t(2 MeV)), log-uniform grids, isotropic 2 MeV
    point source, 50-bin energy flux tally (the C1 set-up with a larger
    material)."""
    rng = np.random.default_rng(data_seed)
    awrs = np.concatenate([[1.0], rng.uniform(2.0, 240.0, n_nuclides - 1)])
    nucs = [make_nuclide(rng, float(a), n_points, "loguniform") for a in awrs]
    mat = make_material(rng, nucs, np.arange(n_nuclides), 0.5, fixed_fraction=(0, 0.5))
    return Problem(name=f"infinite_{n_nuclides}nuc", nuclides=nucs, materials=[mat],
                   geometry=Geometry(kind=GEOM_INFINITE, material=0),
                   source=Source(kind=SRC_POINT), tally=Tally(TALLY_ENERGY, energy_edges(50)),
                   histories=histories, batches=1, seed=seed)


def c1_constant_problem(sig_c: float, sig_s: float, awr: float = 1.0, density: float = 0.01,
                        seed: int = 11, histories: int = 10_000, batches: int = 10,
                        n_bins: int = 50) -> Problem:
    """Infinite medium of one nuclide with constant cross sections (closed-form variant)."""
    nuc = constant_nuclide(sig_c, sig_s, awr)
    mat = Material(nuclides=np.array([0], np.int32), densities=np.array([density]))
    return Problem(name="c1_constant", nuclides=[nuc], materials=[mat],
                   geometry=Geometry(kind=GEOM_INFINITE, material=0),
                   source=Source(kind=SRC_POINT), tally=Tally(TALLY_ENERGY, energy_edges(n_bins)),
                   histories=histories, batches=batches, seed=seed)


PIN_R = 0.41
PIN_PITCH = 1.26


def _lattice_geometry(n: int, pin_mat: np.ndarray, mod_mat: int, height: float = 1.0) -> Geometry:
    return Geometry(kind=GEOM_LATTICE, nx=n, ny=n, pitch=PIN_PITCH, radius=PIN_R, z0=0.0,
                    z1=height, pin_material=pin_mat.astype(np.int32), moderator_material=mod_mat,
                    bc=(BC_REFLECT,) * 6)


def c2_problem(data_seed: int = 2002, seed: int = 2, histories: int = 1_000_000,
               batches: int = 20, grid_range=(10_000, 60_000)) -> Problem:
    """17x17 lattice of cylindrical pins (r 0.41 cm, pitch 1.26 cm, height 1 cm, reflective on
    every face); materials A (30 nuclides, fuel pins), B (3 nuclides, the 25 pins at
    (i, j) in {2,5,8,11,14}^2) and C (5 nuclides, moderator outside every cylinder; its first
    nuclide has A = 1); 38 distinct nuclides on clustered grids of U[10k, 60k] points;
    uniform isotropic 2 MeV source over the box; per-pin track-length flux tally."""
    rng = np.random.default_rng(data_seed)
    n_a, n_b, n_c = 30, 3, 5
    awr = np.concatenate([rng.uniform(2.0, 240.0, n_a + n_b), [1.0], rng.uniform(2.0, 30.0, n_c - 1)])
    sizes = rng.integers(grid_range[0], grid_range[1] + 1, awr.size)
    nucs = [make_nuclide(rng, a, int(s), "clustered") for a, s in zip(awr, sizes)]
    mat_a = make_material(rng, nucs, np.arange(0, n_a), 0.6)
    mat_b = make_material(rng, nucs, np.arange(n_a, n_a + n_b), 0.4)
    mat_c = make_material(rng, nucs, np.arange(n_a + n_b, n_a + n_b + n_c), 0.5,
                          fixed_fraction=(0, 0.6))
    n = 17
    pin = np.zeros((n, n), np.int32)
    for j in (2, 5, 8, 11, 14):
        for i in (2, 5, 8, 11, 14):
            pin[j, i] = 1
    geom = _lattice_geometry(n, pin.ravel(), 2)
    L = n * PIN_PITCH
    return Problem(name="c2_pin_lattice_17x17", nuclides=nucs, materials=[mat_a, mat_b, mat_c],
                   geometry=geom, source=Source(kind=SRC_BOX, box=(0.0, L, 0.0, L, 0.0, 1.0)),
                   tally=Tally(TALLY_PIN), histories=histories, batches=batches, seed=seed)


def assembly_pin_map(core, layouts, pins: int = 17) -> np.ndarray:
    """Pin-cell material map of a core of assemblies, as the flat lattice
    describes it: core[J][I] is the type of the assembly in column I and row
    J (I along x, J along y), layouts[type] a pins x pins array (row j along
    y, column i along x) of pin materials, -1 for a position without a
    cylinder (a water hole or guide tube).  Cell (I*pins + i, J*pins + j)
    of the (NA*pins)^2 lattice takes layouts[core[J][I]][j][i]; the result
    is row-major in y (index y*nx + x), the order of pin_material."""
    core = np.asarray(core, np.int32)
    na_y, na_x = core.shape
    out = np.empty((na_y * pins, na_x * pins), np.int32)
    for J in range(na_y):
        for I in range(na_x):
            lay = np.asarray(layouts[int(core[J, I])], np.int32)
            assert lay.shape == (pins, pins)
            out[J * pins:(J + 1) * pins, I * pins:(I + 1) * pins] = lay
    return out.ravel()


# 17x17 positions of the 24 guide tubes and the central instrument tube of a
# PWR-style assembly (five rows of the symmetric pattern)
GUIDE_TUBES_17 = [(2, 5), (2, 8), (2, 11), (3, 3), (3, 13), (5, 2), (5, 5), (5, 8), (5, 11), (5, 14),
                  (8, 2), (8, 5), (8, 8), (8, 11), (8, 14), (11, 2), (11, 5), (11, 8), (11, 11), (11, 14),
                  (13, 3), (13, 13), (14, 5), (14, 8), (14, 11)]


def core_problem(data_seed: int = 3103, seed: int = 31, histories: int = 200_000,
                 batches: int = 10) -> Problem:
    """A 3x3 core of 17x17-pin assemblies of three types, the flat 51x51
    lattice of the same pins (r 0.41, pitch 1.26, 1 cm high, reflective):
    type 0 fuel (material 0, 20 nuclides) with its 25 guide-tube positions
    empty (water), type 1 the same with absorber rods (material 1, 3
    nuclides) in the guide tubes, type 2 a water assembly (no cylinders).
    Core map (rows along y): [[0, 1, 0], [1, 2, 1], [0, 1, 0]]; moderator
    material 2 (5 nuclides, the first with A = 1); uniform 2 MeV source over
    the box; a 51x51x1 mesh flux tally whose cells are the pin cells."""
    rng = np.random.default_rng(data_seed)
    n_f, n_a, n_m = 20, 3, 5
    awr = np.concatenate([rng.uniform(2.0, 240.0, n_f + n_a), [1.0], rng.uniform(2.0, 30.0, n_m - 1)])
    sizes = rng.integers(5_000, 20_001, awr.size)
    nucs = [make_nuclide(rng, a, int(s), "clustered") for a, s in zip(awr, sizes)]
    fuel = make_material(rng, nucs, np.arange(0, n_f), 0.6)
    absorber = make_material(rng, nucs, np.arange(n_f, n_f + n_a), 0.9)
    moder = make_material(rng, nucs, np.arange(n_f + n_a, n_f + n_a + n_m), 0.5, fixed_fraction=(0, 0.6))
    pins = 17
    t0 = np.zeros((pins, pins), np.int32)
    for j, i in GUIDE_TUBES_17:
        t0[j, i] = -1
    t1 = t0.copy()
    for j, i in GUIDE_TUBES_17:
        t1[j, i] = 1
    t2 = np.full((pins, pins), -1, np.int32)
    core = [[0, 1, 0], [1, 2, 1], [0, 1, 0]]
    n = 3 * pins
    geom = _lattice_geometry(n, assembly_pin_map(core, [t0, t1, t2], pins), 2)
    L = n * PIN_PITCH
    return Problem(name="core_3x3_assemblies", nuclides=nucs, materials=[fuel, absorber, moder],
                   geometry=geom, source=Source(kind=SRC_BOX, box=(0.0, L, 0.0, L, 0.0, 1.0)),
                   tally=Tally(TALLY_MESH, mesh_dims=(n, n, 1), mesh_box=(0.0, L, 0.0, L, 0.0, 1.0)),
                   histories=histories, batches=batches, seed=seed)


def lattice_homogeneous_problem(nuclides: List[Nuclide], material: Material, n: int = 17,
                                seed: int = 21, histories: int = 20_000, batches: int = 10,
                                height: float = 1.0) -> Problem:
    """The 17x17 pin lattice with one material everywhere (closed-form variant)."""
    geom = _lattice_geometry(n, np.zeros(n * n, np.int32), 0, height)
    L = n * PIN_PITCH
    return Problem(name="lattice_homogeneous", nuclides=nuclides, materials=[material],
                   geometry=geom, source=Source(kind=SRC_BOX, box=(0.0, L, 0.0, L, 0.0, height)),
                   tally=Tally(TALLY_PIN), histories=histories, batches=batches, seed=seed)


def c3_problem(data_seed: int = 3003, seed: int = 3, histories: int = 20_000_000,
               batches: int = 1, n_nuclides: int = 300, grid_range=(20_000, 150_000)) -> Problem:
    """15x15 assemblies of 17x17 pins (a 255x255 pin lattice, 321.3 cm square, 1 cm high,
    reflective), one material of 300 nuclides on clustered grids of U[20k, 150k] points,
    uniform isotropic 2 MeV source, 100x100x10 mesh flux tally."""
    rng = np.random.default_rng(data_seed)
    awr = np.concatenate([[1.0], rng.uniform(2.0, 240.0, n_nuclides - 1)])
    sizes = rng.integers(grid_range[0], grid_range[1] + 1, n_nuclides)
    nucs = [make_nuclide(rng, a, int(s), "clustered") for a, s in zip(awr, sizes)]
    mat = make_material(rng, nucs, np.arange(n_nuclides), 0.6, fixed_fraction=(0, 0.4))
    n = 15 * 17
    geom = _lattice_geometry(n, np.zeros(n * n, np.int32), 0)
    L = n * PIN_PITCH
    return Problem(name="c3_assembly_lattice_300nuc", nuclides=nucs, materials=[mat],
                   geometry=geom, source=Source(kind=SRC_BOX, box=(0.0, L, 0.0, L, 0.0, 1.0)),
                   tally=Tally(TALLY_MESH, mesh_dims=(100, 100, 10), mesh_box=(0.0, L, 0.0, L, 0.0, 1.0)),
                   histories=histories, batches=batches, seed=seed)


def slab_problem(sigma_t=(0.2, 1.5, 0.5), thickness=(60.0, 80.0, 40.0 + 20.0),
                 scatter_ratio=(0.0, 0.0, 0.0), awr: float = 1.0, seed: int = 5,
                 histories: int = 100_000, batches: int = 10) -> Problem:
    """Slab of layers along x with constant cross sections, a normally incident 2 MeV beam at
    x = 0 and vacuum on both faces (transmission = weight leaking through the far face)."""
    nucs, mats = [], []
    for k, (st, c) in enumerate(zip(sigma_t, scatter_ratio)):
        nucs.append(constant_nuclide(sig_c=(1.0 - c) * st / 0.01, sig_s=c * st / 0.01, awr=awr))
        mats.append(Material(nuclides=np.array([k], np.int32), densities=np.array([0.01])))
    edges = np.concatenate([[0.0], np.cumsum(thickness)]).astype(np.float64)
    geom = Geometry(kind=GEOM_SLAB, x_edges=edges, layer_material=np.arange(len(sigma_t), dtype=np.int32),
                    bc=(BC_VACUUM, BC_VACUUM, BC_REFLECT, BC_REFLECT, BC_REFLECT, BC_REFLECT))
    return Problem(name="slab", nuclides=nucs, materials=mats, geometry=geom,
                   source=Source(kind=SRC_BEAM, position=(0.0, 0.0, 0.0), direction=(1.0, 0.0, 0.0)),
                   tally=Tally(TALLY_SLAB), histories=histories, batches=batches, seed=seed)


def c4_problem_set(data_seed: int = 4004, seed: int = 4, n_problems: int = 64,
                   histories_range=(1_000, 100_000), nuclide_range=(2, 80),
                   grid_range=(2_000, 10_000)) -> List[Problem]:
    """Independent fixed-source problems of uneven size: histories log-uniform
    in [1e3, 1e5], 2-80 synthetic nuclides (the first with A = 1), clustered
    grids of 2k-10k points, half infinite media (one material, isotropic 2 MeV
    point source) and half single reflective pin cells (r 0.41, pitch 1.26,
    height 1; fuel in the cylinder, the first one or two nuclides as
    moderator outside; uniform source), each with a 50-bin log-energy flux
    tally and its own Philox key (seed << 32 | problem index)."""
    rng = np.random.default_rng(data_seed)
    probs = []
    for p in range(n_problems):
        hist = int(round(_log_uniform(rng, *histories_range)))
        n_nuc = int(rng.integers(nuclide_range[0], nuclide_range[1] + 1))
        awr = np.concatenate([[1.0], rng.uniform(2.0, 240.0, n_nuc - 1)])
        sizes = rng.integers(grid_range[0], grid_range[1] + 1, n_nuc)
        nucs = [make_nuclide(rng, a, int(s), "clustered") for a, s in zip(awr, sizes)]
        key = (seed << 32) | p
        if p % 2 == 0:
            mat = make_material(rng, nucs, np.arange(n_nuc), 0.5, fixed_fraction=(0, 0.5))
            probs.append(Problem(name=f"c4_{p}_infinite", nuclides=nucs, materials=[mat],
                                 geometry=Geometry(kind=GEOM_INFINITE, material=0),
                                 source=Source(kind=SRC_POINT), tally=Tally(TALLY_ENERGY, energy_edges(50)),
                                 histories=hist, batches=1, seed=key))
        else:
            n_mod = 1 if n_nuc == 2 else 2
            mod = make_material(rng, nucs, np.arange(n_mod), 0.5, fixed_fraction=(0, 0.8) if n_mod == 2 else None)
            fuel = make_material(rng, nucs, np.arange(n_mod, n_nuc), 0.6)
            geom = _lattice_geometry(1, np.zeros(1, np.int32), 1)
            probs.append(Problem(name=f"c4_{p}_pincell", nuclides=nucs, materials=[fuel, mod], geometry=geom,
                                 source=Source(kind=SRC_BOX, box=(0.0, PIN_PITCH, 0.0, PIN_PITCH, 0.0, 1.0)),
                                 tally=Tally(TALLY_ENERGY, energy_edges(50)), histories=hist, batches=1,
                                 seed=key))
    return probs


def c5_problem(data_seed: int = 5005, seed: int = 5, histories: int = 10_000_000, batches: int = 20,
               thickness=(100.0, 10.0, 90.0), sigma_t=(0.2, 1.5, 0.2), capture_ratio=(0.005, 0.01, 0.005),
               generator_capture_scale: float = 0.01,
               awr=((56.0, 90.0, 120.0), (184.0, 207.0, 238.0, 56.0), (12.0, 56.0, 120.0)),
               grid_range=(5_000, 20_000)) -> Problem:
    """Deep-penetration slab, x in [0, 200] cm, infinite in y and z: three layers of synthetic
    absorber/scatterer, 100 / 10 / 90 cm thick with Sigma_t(2 MeV) = 0.2 / 1.5 / 0.2 per cm
    (a heavy scatterer, a dense shield, a scatterer with a light component), 53 mean free
    paths at the source energy.  Each layer mixes synthetic nuclides (clustered grids of
    U[5k, 20k] points) whose generated capture is scaled by generator_capture_scale and
    raised by a constant so that capture is capture_ratio[k] of each nuclide's cross
    section at 2 MeV.  With these defaults the analog transmission is about 4e-5 (a few
    hundred scoring histories in 1e7).  A normally incident 2 MeV beam enters at x = 0;
    both x faces are vacuum (the detector is the weight leaking through x = 200); flux
    tally per layer."""
    rng = np.random.default_rng(data_seed)
    nucs, mats = [], []
    for k in range(3):
        first = len(nucs)
        for a in awr[k]:
            nuc = make_nuclide(rng, float(a), int(rng.integers(grid_range[0], grid_range[1] + 1)), "clustered")
            st2 = _analytic_sigma_t(nuc, SOURCE_ENERGY)
            p = float(capture_ratio[k])
            nuc.sig_c = generator_capture_scale * nuc.sig_c + p / (1.0 - p) * st2
            nucs.append(nuc)
        mats.append(make_material(rng, nucs, np.arange(first, len(nucs)), sigma_t[k], density_range=(1e-4, 1e-2)))
    edges = np.concatenate([[0.0], np.cumsum(thickness)]).astype(np.float64)
    geom = Geometry(kind=GEOM_SLAB, x_edges=edges, layer_material=np.arange(3, dtype=np.int32),
                    bc=(BC_VACUUM, BC_VACUUM, BC_REFLECT, BC_REFLECT, BC_REFLECT, BC_REFLECT))
    return Problem(name="c5_deep_penetration_slab", nuclides=nucs, materials=mats, geometry=geom,
                   source=Source(kind=SRC_BEAM, position=(0.0, 0.0, 0.0), direction=(1.0, 0.0, 0.0)),
                   tally=Tally(TALLY_SLAB), histories=histories, batches=batches, seed=seed)


def c5_shield_problem(data_seed: int = 5005, seed: int = 6, histories: int = 4_000_000,
                      batches: int = 20) -> Problem:
    """The deep-penetration slab's recipe with the attenuation concentrated in a
    thin dense shield deep inside: 160 / 12 / 28 cm with Sigma_t(2 MeV) = 0.05 /
    3.0 / 0.05 per cm (8 + 36 + 1.4 mean free paths).  The importance then is
    nearly flat in the first layer and falls steeply across the shield, a shape
    a map linear in depth cannot follow.  Analog transmission about 8e-5."""
    prob = c5_problem(data_seed=data_seed, seed=seed, histories=histories, batches=batches,
                      thickness=(160.0, 12.0, 28.0), sigma_t=(0.05, 3.0, 0.05))
    prob.name = "c5_shielded_slab"
    return prob


def lookup_energies(rng, n: int) -> np.ndarray:
    """Energies log-uniform over [EMIN, EMAX] (the lookup benchmark's input)."""
    return _log_uniform(rng, EMIN, EMAX, n).astype(np.float64)


def edge_case_energies(nuc: Nuclide, rng, n_random: int = 1000) -> np.ndarray:
    """Grid points, their neighbours one ulp away, both ends, and random log-uniform energies."""
    E = nuc.E
    pts = [E, np.nextafter(E, 0.0), np.nextafter(E, np.inf), [EMIN, EMAX],
           lookup_energies(rng, n_random)]
    out = np.concatenate(pts)
    return out[(out >= EMIN) & (out <= EMAX)].astype(np.float64)
