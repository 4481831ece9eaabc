"""The batched solve (vd_batch_*): several uneven lattices advanced by one
launch per schedule step.  Each lattice's arithmetic is that of its own
single-lattice solve (same tiles, same per-lattice reduction order), so the
batch must reproduce the individual solves bit for bit, and match the oracle's
replica solve."""

import numpy as np
import pytest

import oracle
from synth.scenes import make_batch_lattice

from helpers import make_lattice, rotation_angle

pytestmark = pytest.mark.gpu

SIZES = [(12, 3000, 40), (21, 6000, 80), (17, 2500, 30), (30, 9000, 120), (14, 4000, 60)]


def _scenes(gn=3, pcg=8):
    return [make_batch_lattice(500 + k, n, v, s, gn=gn, pcg=pcg)
            for k, (n, v, s) in enumerate(SIZES)]


@pytest.mark.parametrize("tile", [1, 2, 4, 5, 7])
def test_batch_equals_individual_solves(tile):
    from paper_1603_08161_amd import Batch
    scenes = _scenes()
    kw = {"tiles": (tile, tile, tile)}
    lats = [make_lattice(s, **kw) for s in scenes]
    batch = Batch(lats)
    E_batch = batch.solve(reset=True, energies=True)
    for s, lat, e in zip(scenes, lats, E_batch):
        ref = make_lattice(s, **kw)
        rep = ref.solve_frame(reset=True, report=True)
        np.testing.assert_array_equal(e, rep["energy"])
        np.testing.assert_array_equal(lat.get_state()[0], ref.get_state()[0])
        np.testing.assert_array_equal(lat.get_energy(), rep["energy"])


@pytest.mark.parametrize("tile", [0, 7])
def test_batch_equals_individual_solves_fp64(tile):
    """The all-float64 mode through the batched launches (the register-lean
    CG form at the finest level) against single-lattice solves, bitwise."""
    from paper_1603_08161_amd import Batch
    scenes = _scenes(gn=2, pcg=6)[:3]
    kw = {"precision": "fp64", "tiles": (tile, tile, tile)}
    lats = [make_lattice(s, **kw) for s in scenes]
    E_batch = Batch(lats).solve(reset=True, energies=True)
    for s, lat, e in zip(scenes, lats, E_batch):
        ref = make_lattice(s, **kw)
        rep = ref.solve_frame(reset=True, report=True)
        np.testing.assert_array_equal(e, rep["energy"])
        np.testing.assert_array_equal(lat.get_state()[0], ref.get_state()[0])


def test_batch_matches_oracle():
    from paper_1603_08161_amd import Batch
    scenes = _scenes()
    lats = [make_lattice(s) for s in scenes]
    E = Batch(lats).solve(reset=True, energies=True)
    for k in (0, 3):
        ref = oracle.solve_frame(scenes[k])
        assert abs(E[k][0] / ref["energy"][0] - 1.0) < 1e-4
        pos, rot = lats[k].get_state()
        assert np.abs(pos - ref["t"]).max() / scenes[k].spec.spacing < 1e-3
        assert rotation_angle(rot, ref["R"]).max() < 1e-2


def test_batch_graph_replay_equals_eager_and_sequence():
    from paper_1603_08161_amd import Batch
    scenes = _scenes(gn=2, pcg=6)
    eager = [make_lattice(s) for s in scenes]
    graph = [make_lattice(s, graph=True) for s in scenes]
    be, bg = Batch(eager), Batch(graph)
    for frame in range(3):
        # frame 0 from rest, later frames continue from the previous state
        e1 = be.solve(reset=(frame == 0), energies=True)
        e2 = bg.solve(reset=(frame == 0), energies=True)
        np.testing.assert_array_equal(e1, e2)
    for a, b in zip(eager, graph):
        np.testing.assert_array_equal(a.get_state()[0], b.get_state()[0])


def test_batch_rejects_mismatched_handles():
    from paper_1603_08161_amd import Batch, VDError, VD_EINVAL, Lattice
    scenes = _scenes()
    a = make_lattice(scenes[0])
    b = make_lattice(make_batch_lattice(77, 12, 2000, 20, gn=4, pcg=8))  # other schedule
    with pytest.raises(VDError) as ei:
        Batch([a, b])
    assert ei.value.code == VD_EINVAL
    c = make_lattice(scenes[1], graph=True)  # other launch mode
    with pytest.raises(VDError) as ei:
        Batch([a, c])
    assert ei.value.code == VD_EINVAL


@pytest.mark.parametrize("graph", [False, True])
def test_mixed_precision_batch_equals_individual_solves(graph):
    """float32 and float64 lattices in one batch: two parts, the float64 one
    on a forked stream; every lattice bitwise equal to its own solve, the
    energies returned in the caller's order."""
    from paper_1603_08161_amd import Batch
    scenes = _scenes(gn=2, pcg=6)
    precs = ["fp32", "fp64", "fp32", "fp64", "fp64"]
    lats = [make_lattice(s, precision=p, graph=graph) for s, p in zip(scenes, precs)]
    batch = Batch(lats)
    for frame in range(2):
        E = batch.solve(reset=(frame == 0), energies=True)
    for s, p, lat, e in zip(scenes, precs, lats, E):
        ref = make_lattice(s, precision=p, graph=graph)
        ref.solve_frame(reset=True)
        rep = ref.solve_frame(report=True)
        np.testing.assert_array_equal(e, rep["energy"])
        np.testing.assert_array_equal(lat.get_state()[0], ref.get_state()[0])


@pytest.mark.parametrize("graph", [False, True])
def test_batch_tuner_keeps_the_state_and_the_bits(graph):
    """vd_batch_tune (mixed precisions): the state is unchanged by tuning, the
    chosen tiles are set on every handle of a part, and the tuned batch still
    equals single solves with those tiles bit for bit."""
    from paper_1603_08161_amd import Batch
    from paper_1603_08161_amd._lib import VD_TILE_KINDS
    scenes = _scenes(gn=2, pcg=6)
    precs = ["fp64" if k % 2 else "fp32" for k in range(len(scenes))]
    lats = [make_lattice(s, precision=p, graph=graph) for s, p in zip(scenes, precs)]
    batch = Batch(lats)
    batch.solve(reset=True)
    before = [lat.get_state() for lat in lats]
    tiles, us = batch.tune(iters=4)
    print("tuned tiles", tiles, "us/iteration fp32 finest", us[0, 2, :])
    assert set(tiles) == {"fp32", "fp64"}
    for name in tiles:
        assert len(tiles[name]) == 3 and all(1 <= t <= VD_TILE_KINDS for t in tiles[name])
    assert np.all(us[0, :3] > 0) and np.all(us[1, :3] > 0)
    for lat, (p0, r0) in zip(lats, before):
        p1, r1 = lat.get_state()
        np.testing.assert_array_equal(p1, p0)
        np.testing.assert_array_equal(r1, r0)
    E = batch.solve(reset=True, energies=True)
    for s, p, lat, e in zip(scenes, precs, lats, E):
        ref = make_lattice(s, precision=p, tiles=tuple(tiles[p]))
        rep = ref.solve_frame(reset=True, report=True)
        np.testing.assert_array_equal(e, rep["energy"])
        np.testing.assert_array_equal(lat.get_state()[0], ref.get_state()[0])
