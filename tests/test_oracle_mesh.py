"""Pins for the oracle's mesh track-length tally (3-D walk of each flight
through the mesh cells).

* The pieces of every flight add up to the flight: over a mesh that covers
  the whole geometry, the mesh sums equal the total track length (rounding).
* One material everywhere, uniform source, reflective faces: the flux is
  flat, so the expected track length per cell is (1/Sigma_a) V_cell / V.
"""
import numpy as np

import mcsynth
import oracle
from tests.stats import three_sigma


def mesh_problem(n=5, dims=(4, 4, 2), histories=5000):
    nuc = mcsynth.constant_nuclide(10.0, 40.0, 56.0)
    mat = mcsynth.Material(nuclides=np.array([0], np.int32), densities=np.array([0.01]))
    prob = mcsynth.lattice_homogeneous_problem([nuc], mat, n=n, histories=histories)
    L = n * mcsynth.PIN_PITCH
    prob.tally = mcsynth.Tally(mcsynth.TALLY_MESH, mesh_dims=dims, mesh_box=(0.0, L, 0.0, L, 0.0, 1.0))
    return prob


def test_mesh_pieces_add_up_to_the_track_length():
    prob = mesh_problem()
    r = oracle.run(oracle.OracleProblem(prob), 3, 0, 5000)
    assert r.tl.shape == (32,)
    np.testing.assert_allclose(r.tl.sum(), r.glob[oracle.G_TRACK], rtol=1e-11)
    assert np.all(r.tl > 0)


def test_mesh_flux_is_flat_in_a_homogeneous_reflected_box():
    prob = mesh_problem()
    st = oracle.run_batches(oracle.OracleProblem(prob), 5, 20, 5000)
    truth = np.full(32, 10.0 / 32)  # 1/Sigma_a = 10 cm per source particle, equal cell volumes
    n_fail, allowed, z = three_sigma(st.mean["tl"], st.stderr["tl"], truth=truth)
    assert n_fail <= allowed, (n_fail, allowed, z)


def test_partial_mesh_scores_only_inside_its_box():
    """A mesh box over part of the homogeneous reflected lattice: cell c
    expects (1/Sigma_a) V_c / V_geometry, and the cells together hold the
    box's share of the track length, not the whole of it."""
    prob = mesh_problem(dims=(3, 4, 2))
    prob.tally = mcsynth.Tally(mcsynth.TALLY_MESH, mesh_dims=(3, 4, 2), mesh_box=(1.0, 4.0, 0.5, 6.3, 0.25, 0.75))
    st = oracle.run_batches(oracle.OracleProblem(prob), 7, 20, 5000)
    v_cell = (3.0 / 3) * (5.8 / 4) * (0.5 / 2)
    truth = np.full(24, 10.0 * v_cell / (6.3 * 6.3 * 1.0))
    for k in ("tl", "coll"):
        n_fail, allowed, z = three_sigma(st.mean[k], st.stderr[k], truth=truth)
        assert n_fail <= allowed, (k, n_fail, allowed, z)
    share = 3.0 * 5.8 * 0.5 / (6.3 * 6.3)
    assert abs(st.mean["tl"].sum() - 10.0 * share) < 3 * np.sqrt(np.sum(st.stderr["tl"] ** 2))
