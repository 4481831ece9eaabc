"""Precision study on the GPU: the 30-frame deforming sequence on a 96^3
lattice (levels 24^3/48^3/96^3, 8 GN x 20 PCG), each precision mode carried
from its own previous frame, against the FP64 oracle's stored run
(tests/golden/precision_seq96_oracle.npz, written by make_precision_golden.py
from oracle/ only).

Per frame the test records the relative energy error and the largest node
position error (in units of the finest spacing) at the 2048 stored nodes, and
prints the table.  Gates: float32 vectors with float64 reductions stay within
1e-4 relative energy and 1e-3 spacing; the all-float64 mode within 1e-9 and
1e-4 spacing (the stored positions are float32)."""

import os

import numpy as np
import pytest

from synth import make_sequence_frame

from helpers import make_lattice

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "precision_seq96_oracle.npz")


def _run(scenes, precision, idx):
    lat = None
    energies, pos = [], []
    for f, scene in enumerate(scenes):
        if lat is None:
            lat = make_lattice(scene, precision=precision, graph=True)
            lat.solve_frame(reset=True)
        else:
            lat.set_scene(scene)
            lat.solve_frame()
        energies.append(lat.get_energy())
        p, _ = lat.get_state()
        pos.append(p[idx])
    return np.array(energies), np.array(pos)


def test_precision_study_seq96():
    z = np.load(GOLDEN, allow_pickle=False)
    e_ref, p_ref, idx = z["energies"], z["positions"].astype(np.float64), z["node_index"]
    n = int(z["n"])
    frames = e_ref.shape[0]
    assert frames >= 28
    scenes = [make_sequence_frame(int(z["seed"]), f, n=n) for f in range(frames)]
    h = scenes[0].spec.spacing
    rows = {}
    for prec in ("fp32", "fp64"):
        e, p = _run(scenes, prec, idx)
        de = np.abs(e[:, 0] / e_ref[:, 0] - 1.0)
        dx = np.abs(p - p_ref).max(axis=(1, 2)) / h
        rows[prec] = (de, dx)
    print("\nframe  E_oracle        fp32 dE/E  fp32 dx/h  fp64 dE/E  fp64 dx/h")
    for f in range(frames):
        print(f"{f:5d}  {e_ref[f, 0]:.9f}  {rows['fp32'][0][f]:.2e}   {rows['fp32'][1][f]:.2e}"
              f"   {rows['fp64'][0][f]:.2e}   {rows['fp64'][1][f]:.2e}")
    assert rows["fp32"][0].max() < 1e-4
    assert rows["fp32"][1].max() < 1e-3
    assert rows["fp64"][0].max() < 1e-9
    assert rows["fp64"][1].max() < 1e-4
