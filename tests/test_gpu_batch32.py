"""The batched workload at full size: all 32 lattices (24^3 .. 64^3 nodes per
axis, seed 0) solved together from rest, every lattice checked against the
FP64 oracle's replica solve stored by tests/golden/make_batch_golden.py
(final energy within 1e-4 relative; positions at 1024 sampled nodes per
lattice within 1e-3 of the finest spacing), in the graph launch path the
benchmark uses.  Lattices below 33 nodes per axis run in float64 (the
benchmark's precision rule, ``batch_precision``), the others in float32; the
two parts of the batch run concurrently."""

import os

import numpy as np
import pytest

from helpers import make_lattice

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "batch32_oracle.npz")


def _scenes():
    from synth.scenes import make_config2
    return make_config2(0)


@pytest.mark.parametrize("graph", [True])
def test_all_32_lattices_match_oracle(graph):
    from paper_1603_08161_amd import Batch, batch_precision
    gold = np.load(GOLDEN)
    scenes = _scenes()
    assert [s.spec.dims[0] for s in scenes] == list(gold["dims"])
    precs = [batch_precision(s.spec.dims[0]) for s in scenes]
    assert "fp32" in precs and "fp64" in precs
    lats = [make_lattice(s, graph=graph, precision=p) for s, p in zip(scenes, precs)]
    E = Batch(lats).solve(reset=True, energies=True)
    worst = {"fp32": [0.0, 0.0], "fp64": [0.0, 0.0]}
    for k, (s, lat) in enumerate(zip(scenes, lats)):
        e_rel = abs(E[k][0] / gold["energies"][k][0] - 1.0)
        n = s.spec.dims[0] ** 3
        m = min(n, gold["node_index"].shape[1])
        idx = gold["node_index"][k][:m]
        pos = lat.get_state()[0][idx].astype(np.float64)
        dp = float(np.abs(pos - gold["positions"][k][:m]).max() / s.spec.spacing)
        print(f"lattice {k:2d} n={s.spec.dims[0]} {precs[k]}: rel E {e_rel:.2e}, "
              f"max |dt|/h {dp:.2e}")
        w = worst[precs[k]]
        w[0], w[1] = max(w[0], e_rel), max(w[1], dp)
    for p, (we, wp) in worst.items():
        print(f"worst {p}: rel E {we:.3e}, max |dt|/h {wp:.3e}")
    for we, wp in worst.values():
        assert we <= 1e-4
        assert wp <= 1e-3
