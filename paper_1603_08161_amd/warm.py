"""Learned warm start: training data from the plain solver, training on the
GPU through the library's network kernels, and the warm-vs-plain evaluation.

Not part of the paper.  Every frame k >= 2 of a deforming sequence gives one
sample: the input features of vd_warm_features at the previous frame's solved
state (with the frame before as the second displacement) and, as the label,
the change of the node displacements that the plain schedule (Sec. 7) then
produces, in units of the finest spacing.  Sequences are seeded deforming
tori (moving Gaussian RBF warps) rendered to 640x480 depth maps; scenes are
generated on the host by worker processes while the GPU solves.

Run as ``python -m paper_1603_08161_amd.warm --out weights.npz`` (trains and
evaluates) or ``--eval-only --weights weights.npz``.
"""

from __future__ import annotations

import argparse
import multiprocessing as mp
import os
import sys
import time
from typing import Dict, List

import numpy as np

from ._lib import Lattice, Net

WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "warm64.npz")


def _frame_scene(args):
    """Worker: one frame of one seeded sequence (host-only numpy work)."""
    seed, k, n = args
    from synth.scenes import make_sequence_frame
    return make_sequence_frame(seed, k, n=n)


def _one_thread():
    """Worker initialiser: one BLAS/OpenMP thread per worker process, so the
    pool does not oversubscribe the host cores."""
    from threadpoolctl import threadpool_limits
    threadpool_limits(limits=1)


def make_pool(workers: int):
    """Spawned worker processes for scene generation, or None (generate in
    this process).  Create it before the GPU is first used: the workers are
    started by fork + exec."""
    if workers <= 0:
        return None
    return mp.get_context("spawn").Pool(workers, initializer=_one_thread)


def sequence_pool(pool, seeds, frames, n):
    """Iterator over (seed, scenes) in seed order; the frames are generated in
    parallel across the pool's workers."""
    jobs = [(s, k, n) for s in seeds for k in range(frames)]
    it = map(_frame_scene, jobs) if pool is None else pool.imap(_frame_scene, jobs)
    for s in seeds:
        yield s, [next(it) for _ in range(frames)]


class SequenceRunner:
    """One lattice replaying sequences with the plain schedule (hipGraph)."""

    def __init__(self, scene0):
        self.lat = Lattice.from_spec(scene0.spec, graph=True)
        self.spec = scene0.spec
        g = self.spec
        nx, ny, nz = g.dims
        a = np.arange(nx * ny * nz)
        idx = np.stack([a % nx, (a // nx) % ny, a // (nx * ny)], axis=1)
        self.rest = (np.asarray(g.origin)[None, :] + g.spacing * idx).astype(np.float64)
        self.n = nx * ny * nz
        self.h = g.spacing

    def disp(self) -> np.ndarray:
        """Current finest displacement t - t_hat as [3][N] float32."""
        pos, _ = self.lat.get_state()
        return (pos.astype(np.float64) - self.rest).T.astype(np.float32).copy()


def sequence_samples(runner: "SequenceRunner", scenes, X, Y, i0: int, device) -> int:
    """Solve one sequence with the plain schedule and write the samples of its
    frames 2.. into X[i0:], Y[i0:]; returns the next free index."""
    import torch
    lat = runner.lat
    lat.set_scene(scenes[0])
    lat.solve_frame(reset=True)
    d_prev2 = runner.disp()
    lat.set_scene(scenes[1])
    lat.solve_frame()
    d_prev = runner.disp()
    i = i0
    for k in range(2, len(scenes)):
        lat.set_scene(scenes[k])
        lat.warm_features(prev2=torch.from_numpy(d_prev2).to(device), out=X[i])
        lat.solve_frame()
        d = runner.disp()
        Y[i].copy_(torch.from_numpy(((d - d_prev) / runner.h).reshape(-1)))
        d_prev2, d_prev = d_prev, d
        i += 1
    return i


def build_dataset(pool, seeds, frames, n, device, log=print):
    """Features X [F][8N] (int16 bfloat16 bits) and labels Y [F][3N] (float32)
    on `device` for frames 2..frames-1 of every sequence."""
    import torch
    X = Y = None
    runner = None
    i = 0
    t0 = time.time()
    for seed, scenes in sequence_pool(pool, seeds, frames, n):
        if runner is None:
            runner = SequenceRunner(scenes[0])
            X = torch.empty((len(seeds) * (frames - 2), 8 * runner.n), dtype=torch.int16,
                            device=device)
            Y = torch.empty((len(seeds) * (frames - 2), 3 * runner.n), dtype=torch.float32,
                            device=device)
        i = sequence_samples(runner, scenes, X, Y, i, device)
        log(f"# data: sequence {seed} done ({i} samples, {time.time() - t0:.0f} s)")
    return X, Y


def init_params(seed: int = 0, head_scale: float = 0.1) -> np.ndarray:
    """He-normal weights (std sqrt(2 / fan_in)), zero biases, a small head so
    the untrained network predicts almost no change; vd_net.h order."""
    rng = np.random.default_rng(seed)
    layers = [(8, 16), (16, 16), (16, 32), (32, 32), (32, 64), (64, 64), (64, 32), (64, 32),
              (32, 16), (32, 16), (16, 3)]
    out = []
    for li, (ci, co) in enumerate(layers):
        std = np.sqrt(2.0 / (27 * ci)) * (head_scale if li == len(layers) - 1 else 1.0)
        out.append(rng.normal(scale=std, size=co * ci * 27))
        out.append(np.zeros(co))
    return np.concatenate(out).astype(np.float32)


class Trainer:
    """Adam on random mini-batches drawn from the first `count` samples."""

    def __init__(self, net: Net, X, Y, batch: int, lr: float, seed: int = 0, log=print):
        import torch
        self.net, self.X, self.Y, self.batch, self.lr, self.log = net, X, Y, batch, lr, log
        self.rng = np.random.default_rng(seed)
        self.xb = torch.empty((batch, X.shape[1]), dtype=X.dtype, device=X.device)
        self.yb = torch.empty((batch, Y.shape[1]), dtype=Y.dtype, device=Y.device)
        self.step = 0
        self.curve = []
        self.t0 = time.time()

    def run(self, steps: int, count: int) -> None:
        import torch
        for _ in range(steps):
            idx = torch.from_numpy(self.rng.integers(0, count, size=self.batch)).to(self.X.device)
            torch.index_select(self.X, 0, idx, out=self.xb)
            torch.index_select(self.Y, 0, idx, out=self.yb)
            want = self.step % 100 == 0
            loss = self.net.train_step(self.xb, self.yb, batch=self.batch, lr=self.lr,
                                       want_loss=want)
            if want:
                self.curve.append((self.step, loss))
                self.log(f"# train step {self.step}: loss {loss:.5f} on {count} samples "
                         f"({time.time() - self.t0:.0f} s)")
            self.step += 1


def train_streaming(net: Net, pool, seeds, frames, n, device, steps_per_seq: int,
                    final_steps: int, batch: int, lr: float, out: str, meta: Dict,
                    log=print):
    """Generate, solve and train in one pass: after each sequence arrives its
    samples join the data set and `steps_per_seq` Adam steps run over all
    samples so far (the workers meanwhile generate the next sequences); then
    `final_steps` more.  The weights are saved after every 5 sequences and at
    the end."""
    import torch
    X = Y = None
    runner = trainer = None
    i = 0
    t0 = time.time()
    for j, (seed, scenes) in enumerate(sequence_pool(pool, seeds, frames, n)):
        if runner is None:
            runner = SequenceRunner(scenes[0])
            X = torch.empty((len(seeds) * (frames - 2), 8 * runner.n), dtype=torch.int16,
                            device=device)
            Y = torch.empty((len(seeds) * (frames - 2), 3 * runner.n), dtype=torch.float32,
                            device=device)
            trainer = Trainer(net, X, Y, batch, lr, log=log)
        i = sequence_samples(runner, scenes, X, Y, i, device)
        log(f"# data: sequence {seed} done ({i} samples, {time.time() - t0:.0f} s)")
        trainer.run(steps_per_seq, i)
        if (j + 1) % 5 == 0:
            save_weights(out, net.get_params(), dict(meta, sequences=j + 1, steps=trainer.step,
                                                     curve=trainer.curve))
    trainer.run(final_steps, i)
    rms = float(Y[:i].pow(2).mean().sqrt())
    save_weights(out, net.get_params(), dict(meta, sequences=len(seeds), steps=trainer.step,
                                             curve=trainer.curve, label_rms=rms))
    log(f"# train: {trainer.step} steps over {i} samples (label rms {rms:.4f} voxel) in "
        f"{time.time() - t0:.0f} s; saved {out}")
    return trainer.curve


def evaluate(net: Net, pool, seeds, frames, n, device, max_gn: int = 16, log=print) -> Dict:
    """Per held-out frame k >= 2, from the plain chain's state t^{k-1}:
    the plain schedule (time, energy E_plain), then finest-level iterations
    until E <= E_plain from (a) the judged network prediction and (b) the plain
    initialisation.  Returns per-frame records and their means."""
    import torch
    recs: List[Dict] = []
    runner = None
    sync = torch.cuda.synchronize
    for seed, scenes in sequence_pool(pool, seeds, frames, n):
        if runner is None:
            runner = SequenceRunner(scenes[0])
            out = torch.empty(3 * runner.n, dtype=torch.float32, device=device)
            cv = torch.empty(3 * runner.n, dtype=torch.float32, device=device)
            xbuf = torch.empty(8 * runner.n, dtype=torch.int16, device=device)
            rest_t = torch.from_numpy(runner.rest.T.astype(np.float32).copy()).to(device)

            def lab_dev(pos, d_last=None):
                """Solved displacement change (pos - t^{k-1}) / h as [3N]."""
                dp = torch.from_numpy(pos.T.astype(np.float32).copy()).to(device) - rest_t
                return ((dp - torch.from_numpy(d_prev).to(device)) / runner.h).reshape(-1)
        lat = runner.lat
        lat.set_scene(scenes[0])
        lat.solve_frame(reset=True)
        d_prev2 = runner.disp()
        lat.set_scene(scenes[1])
        lat.solve_frame()
        d_prev = runner.disp()
        for k in range(2, frames):
            lat.set_scene(scenes[k])
            pos0, rot0 = lat.get_state()
            p2 = torch.from_numpy(d_prev2).to(device)
            # plain schedule
            sync()
            t = time.perf_counter()
            lat.solve_frame()
            e_plain = float(lat.get_energy()[0])
            t_plain = time.perf_counter() - t
            pos1, rot1 = lat.get_state()
            target = e_plain * (1.0 + 1e-6)
            # (a) network prediction, judged, then finest-level iterations
            lat.set_state(pos0, rot0)
            sync()
            t = time.perf_counter()
            lat.warm_features(prev2=p2, out=xbuf)
            net.forward(xbuf, batch=1, out=out)
            rw = lat.solve_frame(report=True, init_delta=out, energy_target=target,
                                 max_gn=max_gn)
            t_warm = time.perf_counter() - t
            # (b) plain initialisation, same stopping rule
            lat.set_state(pos0, rot0)
            sync()
            t = time.perf_counter()
            rp = lat.solve_frame(report=True, energy_target=target, max_gn=max_gn)
            t_pt = time.perf_counter() - t
            # (c) non-learned baseline: constant-velocity extrapolation of the
            # last two frames, judged the same way
            lat.set_state(pos0, rot0)
            cv.copy_(torch.from_numpy(((d_prev - d_prev2) / runner.h).reshape(-1)))
            rc = lat.solve_frame(report=True, init_delta=cv, energy_target=target,
                                 max_gn=max_gn)
            # (d) the prediction as a direction: the exact minimum of E along
            # it at fixed rotations, judged, same stopping rule
            lat.set_state(pos0, rot0)
            sync()
            t = time.perf_counter()
            lat.warm_features(prev2=p2, out=xbuf)
            net.forward(xbuf, batch=1, out=out)
            rs = lat.solve_frame(report=True, init_delta=out, energy_target=target,
                                 max_gn=max_gn, warm_step=True)
            t_step = time.perf_counter() - t
            net_err = float(((out - lab_dev(pos1)) ** 2).sum() / runner.n)
            recs.append(dict(seed=seed, frame=k, e_plain=e_plain, t_plain_ms=1e3 * t_plain,
                             e_init_plain=rw["init_energy"][0],
                             e_init_warm=rw["init_energy"][1], warm_used=rw["warm_used"],
                             gn_warm=rw["gn_done"], reached_warm=rw["target_reached"],
                             e_warm=float(rw["energy"][0]), t_warm_ms=1e3 * t_warm,
                             gn_plain_target=rp["gn_done"], reached_plain=rp["target_reached"],
                             t_plain_target_ms=1e3 * t_pt, e_plain_target=float(rp["energy"][0]),
                             e_init_cv=rc["init_energy"][1], cv_used=rc["warm_used"],
                             gn_cv=rc["gn_done"], reached_cv=rc["target_reached"],
                             e_init_step=rs["init_energy"][1], step_used=rs["warm_used"],
                             gn_step=rs["gn_done"], reached_step=rs["target_reached"],
                             t_step_ms=1e3 * t_step,
                             pred_mse=net_err,
                             cv_mse=float(((cv - lab_dev(pos1)) ** 2).sum() / runner.n),
                             zero_mse=float((lab_dev(pos1) ** 2).sum() / runner.n)))
            # continue the chain with the plain solution
            lat.set_state(pos1, rot1)
            d = runner.disp()
            d_prev2, d_prev = d_prev, d
        r = recs[-1]
        log(f"# eval: sequence {seed}: last frame E_plain {r['e_plain']:.4f}, "
            f"init warm/plain {r['e_init_warm'] / r['e_init_plain']:.3f}, "
            f"cv/plain {r['e_init_cv'] / r['e_init_plain']:.3f}, "
            f"GN warm {r['gn_warm']} cv {r['gn_cv']} plain-init {r['gn_plain_target']}, "
            f"mse net {r['pred_mse']:.2e} cv {r['cv_mse']:.2e} zero {r['zero_mse']:.2e}")
    return dict(frames=recs, summary=summarise(recs))


def summarise(recs: List[Dict]) -> Dict:
    a = lambda k: np.array([r[k] for r in recs], np.float64)
    return dict(
        frames=len(recs),
        init_energy_ratio_mean=float(np.mean(a("e_init_warm") / a("e_init_plain"))),
        warm_used_frac=float(np.mean(a("warm_used"))),
        warm_reached_frac=float(np.mean(a("reached_warm"))),
        plain_init_reached_frac=float(np.mean(a("reached_plain"))),
        gn_warm_mean=float(np.mean(a("gn_warm"))),
        gn_plain_init_mean=float(np.mean(a("gn_plain_target"))),
        t_plain_ms_mean=float(np.mean(a("t_plain_ms"))),
        t_warm_ms_mean=float(np.mean(a("t_warm_ms"))),
        t_plain_init_target_ms_mean=float(np.mean(a("t_plain_target_ms"))),
        cv_init_energy_ratio_mean=float(np.mean(a("e_init_cv") / a("e_init_plain"))),
        cv_reached_frac=float(np.mean(a("reached_cv"))),
        gn_cv_mean=float(np.mean(a("gn_cv"))),
        pred_mse_mean=float(np.mean(a("pred_mse"))),
        cv_mse_mean=float(np.mean(a("cv_mse"))),
        zero_mse_mean=float(np.mean(a("zero_mse"))),
        # the warm start's own factor: the same stopping rule from the plain
        # initialisation over the judged prediction (> 1: the network helps)
        warm_start_factor=float(np.mean(a("t_plain_target_ms")) / np.mean(a("t_warm_ms"))),
        warm_start_gn_factor=float(np.mean(a("gn_plain_target")) / max(np.mean(a("gn_warm")), 1e-9)),
        # the prediction used as a direction (exact line minimum), judged
        step_init_energy_ratio_mean=float(np.mean(a("e_init_step") / a("e_init_plain"))),
        step_used_frac=float(np.mean(a("step_used"))),
        step_reached_frac=float(np.mean(a("reached_step"))),
        gn_step_mean=float(np.mean(a("gn_step"))),
        t_step_ms_mean=float(np.mean(a("t_step_ms"))),
        warm_step_factor=float(np.mean(a("t_plain_target_ms")) / np.mean(a("t_step_ms"))),
        # the plain schedule over the warm path: credits the energy-target
        # stopping rule as much as the network
        speedup_vs_plain_schedule=float(np.mean(a("t_plain_ms")) / np.mean(a("t_warm_ms"))),
    )


def save_weights(path: str, params: np.ndarray, meta: Dict) -> None:
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    np.savez_compressed(path, params=params.astype(np.float32),
                        meta=np.frombuffer(repr(meta).encode(), np.uint8))


def load_weights(path: str = WEIGHTS) -> np.ndarray:
    with np.load(path, allow_pickle=False) as z:
        return np.asarray(z["params"], np.float32)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--train-seqs", type=int, default=50)
    ap.add_argument("--test-seqs", type=int, default=10)
    ap.add_argument("--frames", type=int, default=40)
    ap.add_argument("--steps-per-seq", type=int, default=50)
    ap.add_argument("--final-steps", type=int, default=500)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--workers", type=int, default=14)
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--weights", default=None)
    ap.add_argument("--eval-only", action="store_true")
    ap.add_argument("--eval-seqs", type=int, default=None)
    ap.add_argument("--report", default=None)
    a = ap.parse_args(argv)
    log = lambda s: print(s, flush=True)
    pool = make_pool(a.workers)  # before the first GPU call
    import torch
    dev = torch.device("cuda:0")
    train_seeds = list(range(a.train_seqs))
    test_seeds = list(range(1000, 1000 + (a.eval_seqs or a.test_seqs)))
    nodes = (a.n, a.n, a.n)
    net = Net(nodes, max_batch=a.batch)
    if a.eval_only:
        net.set_params(load_weights(a.weights or WEIGHTS))
    else:
        net.set_params(init_params(0))
        meta = dict(n=a.n, train_seqs=a.train_seqs, frames=a.frames, batch=a.batch, lr=a.lr)
        train_streaming(net, pool, train_seeds, a.frames, a.n, dev, a.steps_per_seq,
                        a.final_steps, a.batch, a.lr, a.out, meta, log=log)
    res = None
    if a.eval_seqs != 0:
        res = evaluate(net, pool, test_seeds, a.frames, a.n, dev, log=log)
    if pool is not None:
        pool.close()
        pool.join()
    if res is None:
        return 0
    log("# summary " + repr(res["summary"]))
    if a.report:
        import json
        with open(a.report, "w") as f:
            json.dump(res, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
