"""Writes tests/golden/precision_seq96_oracle.npz: the FP64 oracle (replica
mode) on the 30-frame, 96^3 deforming sequence used by the precision study.

Each frame is solved from the previous frame's oracle state (frame 0 from
rest).  Stored per frame: the energy terms of eq. (1) and the final positions
at 2048 seeded node indices (float32; the study's tolerance is 1e-3 of the
spacing).  Calls only synth/ and oracle/.

Usage: python tests/golden/make_precision_golden.py [n_frames]
"""

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from synth import make_sequence_frame  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "precision_seq96_oracle.npz")
SEED = 0
N = 96
N_SAMPLE = 2048


def main():
    frames = int(sys.argv[1]) if len(sys.argv) > 1 else 30
    rng = np.random.default_rng(1234)
    idx = np.sort(rng.choice(N ** 3, size=N_SAMPLE, replace=False))
    energies = np.zeros((frames, 4))
    pos = np.zeros((frames, N_SAMPLE, 3), np.float32)
    state = None
    for f in range(frames):
        t0 = time.time()
        scene = make_sequence_frame(SEED, f, n=N)
        out = oracle.solve_frame(scene, state=state)
        state = (out["t"], out["R"])
        energies[f] = out["energy"]
        pos[f] = out["t"][idx]
        print(f"frame {f}: E = {out['energy'][0]:.9g} ({time.time() - t0:.1f} s)", flush=True)
        np.savez(OUT, energies=energies[: f + 1], positions=pos[: f + 1], node_index=idx,
                 seed=SEED, n=N)


if __name__ == "__main__":
    main()
