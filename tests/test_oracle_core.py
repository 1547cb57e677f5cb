"""A core of assemblies with different pin layouts, as the flat lattice
describes it (no GPU): the map puts each assembly's layout at its place, and
the oracle's geometry reads it that way (positions without a cylinder score
no pin flux, every other pin does)."""
import dataclasses

import numpy as np

import mcsynth
import oracle


def test_assembly_pin_map_places_each_layout():
    rng = np.random.default_rng(5)
    pins = 4
    layouts = [rng.integers(-1, 3, (pins, pins)).astype(np.int32) for _ in range(3)]
    core = [[0, 2], [1, 0], [2, 2]]  # 3 rows along y, 2 columns along x
    flat = mcsynth.assembly_pin_map(core, layouts, pins)
    nx, ny = 2 * pins, 3 * pins
    assert flat.shape == (nx * ny,)
    for J in range(3):
        for I in range(2):
            for j in range(pins):
                for i in range(pins):
                    x, y = I * pins + i, J * pins + j
                    assert flat[y * nx + x] == layouts[core[J][I]][j][i]
    # one assembly: its own layout
    assert np.array_equal(mcsynth.assembly_pin_map([[1]], layouts, pins), layouts[1].ravel())


def test_core_positions_without_cylinder_score_no_pin_flux():
    prob = mcsynth.core_problem()
    mat = prob.geometry.pin_material.reshape(51, 51)
    # 4 fuel assemblies with 25 open guide tubes, 4 with absorber rods in
    # them, a water assembly in the middle
    assert (mat == -1).sum() == 4 * 25 + 289 and (mat == 1).sum() == 4 * 25
    assert np.all(mat[17:34, 17:34] == -1)
    pin = dataclasses.replace(prob, tally=mcsynth.Tally(mcsynth.TALLY_PIN))
    r = oracle.run(oracle.OracleProblem(pin), 31, 0, 20_000)
    tl = r.tl.reshape(51, 51)
    assert np.all(tl[mat == -1] == 0.0)
    assert np.all(tl[mat != -1] > 0.0)
