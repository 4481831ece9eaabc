"""Writes tests/golden/batch32_oracle.npz: the FP64 oracle (replica mode) on
every lattice of the batched workload (32 lattices, 24^3 .. 64^3 nodes per
axis, seed 0 of ``synth.scenes.make_config2``), each solved from rest with its
own 3 levels x 8 GN x 20 PCG schedule.

Stored per lattice: the energy terms of eq. (1) at the final state and the
final positions at 1024 seeded node indices (float32; the gate is 1e-3 of the
spacing).  Calls only synth/ and oracle/.

Usage: python tests/golden/make_batch_golden.py [workers]
"""

import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch32_oracle.npz")
SEED = 0
COUNT = 32
N_SAMPLE = 1024


def sample_index(k: int, n_nodes: int) -> np.ndarray:
    rng = np.random.default_rng(4321 + k)
    return np.sort(rng.choice(n_nodes, size=min(N_SAMPLE, n_nodes), replace=False))


def solve_one(k: int):
    from threadpoolctl import threadpool_limits

    import oracle
    from synth.scenes import make_config2_member
    t0 = time.time()
    scene = make_config2_member(SEED, k)
    with threadpool_limits(limits=1):
        out = oracle.solve_frame(scene)
    n = scene.spec.dims
    idx = sample_index(k, n[0] * n[1] * n[2])
    return k, n[0], out["energy"], out["t"][idx].astype(np.float32), idx, time.time() - t0


def main():
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else 4
    energies = np.zeros((COUNT, 4))
    dims = np.zeros(COUNT, np.int64)
    pos = np.zeros((COUNT, N_SAMPLE, 3), np.float32)
    index = np.zeros((COUNT, N_SAMPLE), np.int64)
    with ProcessPoolExecutor(max_workers=workers) as ex:
        for k, n, e, p, idx, dt in ex.map(solve_one, range(COUNT)):
            energies[k] = e
            dims[k] = n
            pos[k, : p.shape[0]] = p
            index[k, : idx.shape[0]] = idx
            print(f"lattice {k}: n = {n}, E = {e[0]:.9g} ({dt:.1f} s)", flush=True)
    np.savez_compressed(OUT, energies=energies, dims=dims, positions=pos, node_index=index,
                        seed=SEED)


if __name__ == "__main__":
    main()
