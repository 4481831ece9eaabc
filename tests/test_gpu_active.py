"""The solve restricted to the optimised set M (VD_FLAG_ACTIVE_SET; Sec. 6-8)
through the C-ABI against oracle/active.py on the same seeded inputs: the
set itself bit for bit on every level, the frame in float64 and float32, grid
growth between frames, every tile kind and the batched and graph launch
paths bitwise against the single eager solve, and the 64^3 workload."""

import numpy as np
import pytest

from oracle import active
from oracle.energy import prepare_constraints
from oracle.lattice import level_grids
from synth.scenes import make_config1, make_patch

from helpers import make_lattice

pytestmark = pytest.mark.gpu


def _grids_cons(scene):
    s = scene.spec
    grids = level_grids(s.dims, s.spacing, s.origin, s.num_levels)
    return grids, prepare_constraints(scene, grids[0])


def _patch(seed=1, n=20, levels=2, extent=0.6, gn=3, pcg=10):
    return make_patch(seed=seed, dims=(n, n, n), n_dense=2500, n_sparse=20, num_levels=levels,
                      gn=gn, pcg=pcg, extent=extent, amp=0.6)


def test_active_set_matches_oracle_on_every_level():
    sc = _patch()
    grids, cons = _grids_cons(sc)
    lat = make_lattice(sc, active_set=True)
    for lvl, g in enumerate(grids):
        mask, count, _ = lat.get_active(lvl)
        ref = active.active_set(g, cons)
        np.testing.assert_array_equal(mask, ref)
        assert count == int(ref.sum())
        print(f"level {lvl}: |M| = {count} of {g.n}")
    assert 0.05 < lat.get_active(1)[1] / grids[1].n < 0.6


# the float64 mode is compared through the float64 state export
@pytest.mark.parametrize("precision,tol_e,tol_p", [("fp64", 1e-12, 1e-10), ("fp32", 1e-4, 1e-3)])
def test_active_solve_matches_oracle(precision, tol_e, tol_p):
    sc = _patch(seed=2)
    lat = make_lattice(sc, active_set=True, precision=precision)
    rep = lat.solve_frame(reset=True, report=True)
    ref = active.solve_frame_active(sc)
    pos = lat.get_state64()[0]
    e_rel = abs(rep["energy"][0] / ref["energy"][0] - 1.0)
    dp = np.abs(pos - ref["t"]).max() / sc.spec.spacing
    act = ref["active"]
    rest = ref["grid"].rest_positions()
    print(f"{precision}: E gpu {rep['energy'][0]:.9g} oracle {ref['energy'][0]:.9g} rel {e_rel:.2e}, "
          f"max |dt|/h {dp:.2e}, |M| {act.sum()}")
    assert e_rel <= tol_e
    assert dp <= tol_p
    # points outside M stay at rest (the frame started from rest)
    np.testing.assert_allclose(pos[~act], rest[~act], rtol=0, atol=1e-6 * sc.spec.spacing)
    np.testing.assert_allclose(rep["energy"][1:].sum(), rep["energy"][0], rtol=1e-12)


def test_grid_growth_between_frames_matches_oracle():
    """Frame 1 on a small patch, frame 2 on a larger one: the points that
    join M are extrapolated (same layers as the oracle), then solved."""
    small = _patch(seed=3, extent=0.35, n=18)
    big = _patch(seed=3, extent=0.6, n=18)
    lat = make_lattice(small, active_set=True, precision="fp64")
    lat.solve_frame(reset=True)
    r1 = active.solve_frame_active(small)
    lat.set_scene(big)
    _, _, layers = lat.get_active()
    r2 = active.solve_frame_active(big, state=(r1["t"], r1["R"]), prev_active=r1["active"])
    assert layers == r2["layers"] >= 1
    rep = lat.solve_frame(report=True)
    pos = lat.get_state64()[0]
    e_rel = abs(rep["energy"][0] / r2["energy"][0] - 1.0)
    dp = np.abs(pos - r2["t"]).max() / big.spec.spacing
    print(f"growth: {layers} layers, |M| {r1['active'].sum()} -> {r2['active'].sum()}, "
          f"E rel {e_rel:.2e}, max |dt|/h {dp:.2e}")
    assert e_rel <= 1e-12
    assert dp <= 1e-10


def test_every_tile_kind_and_graph_give_the_same_bits():
    sc = _patch(seed=4, n=22)
    ref = make_lattice(sc, active_set=True)
    e_ref = ref.solve_frame(reset=True, report=True)["energy"]
    p_ref = ref.get_state()[0]
    for tile in range(1, 9):
        for graph in (False, True):
            lat = make_lattice(sc, active_set=True, tiles=(tile, tile), graph=graph)
            e = lat.solve_frame(reset=True, report=True)["energy"]
            np.testing.assert_array_equal(e, e_ref)
            np.testing.assert_array_equal(lat.get_state()[0], p_ref)


def test_batched_active_set_equals_single_solves():
    from paper_1603_08161_amd import Batch
    scenes = [_patch(seed=10 + k, n=n) for k, n in enumerate((14, 20, 17))]
    lats = [make_lattice(s, active_set=True) for s in scenes]
    E = Batch(lats).solve(reset=True, energies=True)
    for s, lat, e in zip(scenes, lats, E):
        ref = make_lattice(s, active_set=True)
        rep = ref.solve_frame(reset=True, report=True)
        np.testing.assert_array_equal(e, rep["energy"])
        np.testing.assert_array_equal(lat.get_state()[0], ref.get_state()[0])


def test_active_set_64cubed_matches_oracle():
    """The 64^3 workload restricted to M (3.3 % of the finest points)."""
    sc = make_config1(0)
    lat = make_lattice(sc, active_set=True, graph=True)
    lat.solve_frame(reset=True)
    e = lat.get_energy()
    ref = active.solve_frame_active(sc)
    pos = lat.get_state()[0].astype(np.float64)
    e_rel = abs(e[0] / ref["energy"][0] - 1.0)
    dp = np.abs(pos - ref["t"]).max() / sc.spec.spacing
    _, count, _ = lat.get_active()
    print(f"64^3 active set: |M| {count}, E gpu {e[0]:.9g} oracle {ref['energy'][0]:.9g} "
          f"rel {e_rel:.2e}, max |dt|/h {dp:.2e}")
    assert count == int(ref["active"].sum())
    assert e_rel <= 1e-4
    assert dp <= 1e-3
