"""Benchmark: solved frames/s of the 64^3 lattice solve on one MI355X.

One step = one frame of the hot path on device-resident inputs:
vd_set_constraints (rows, binning, B^T B cache, preconditioner for all three
levels) + vd_solve_frame (3 levels x 8 flip-flop iterations x 20 CG
iterations, from rest) + vd_get_energy.  A frame counts as solved when its
final energy is within 1e-4 relative of the FP64 oracle's replica solve of
the same input.

Also reported:
* roofline -- the fused CG-iteration kernel on the 64^3 level (one launch =
  one Jacobi-PCG iteration): algorithmic bytes per iteration (144 B per node
  + 24 B per dense and 12 B per sparse sample, float32) over its mean
  duration, timed by device clock stamps that the library captures into the
  frame's graph around those launches (read back after the timed replays);
  traffic from the committed rocprofv3 byte-counter summary;
* cpu_baseline -- the FP64 oracle timed on this host on one full frame.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "solved frames/s at 64³ lattice (energy ≤1e-4 of oracle), HBM %; warm vs plain"
HBM_PEAK_GBS = 8000.0
# association thresholds (eps_d in metres, eps_n and eps_v on 1 - cos)
TRACK_EPS = (0.05, 0.3, 0.95)


def cg_iteration_bytes(n_nodes: int, n_dense: int, n_sparse: int, elem: int = 4) -> float:
    """Compulsory bytes of one Jacobi-PCG iteration on a level: 12 node-vector
    passes of 3 components (phase A reads r, D^-1, p and writes p, A p; phase
    B reads d, p, r, A p, D^-1 and writes d, r) plus 24 B per dense and 12 B
    per sparse sample for the data term."""
    return 36.0 * elem * n_nodes + 24.0 * n_dense + 12.0 * n_sparse


def kernel_source_sha() -> str:
    """Hash of the sources the CG-iteration kernel is compiled from."""
    import hashlib
    h = hashlib.sha256()
    for f in ("solve.hip", "vd_device.h", "vd_kernels.h"):
        with open(os.path.join(ROOT, "paper_1603_08161_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(key: str, name: str = "traffic_k_cg_frame64.md"):
    """HBM bytes per launch of a CG-iteration kernel from a committed
    rocprofv3 counter summary (FETCH_SIZE + WRITE_SIZE, scaled by the same
    counters on a plain copy), e.g. key "tile7" for the 64^3 kernel with
    stencil tile 7; None if the summary is missing, has no such entry, or the
    kernel's sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha") != kernel_source_sha():
        return None
    try:
        return float(kv[f"traffic_bytes_per_launch_{key}"])
    except (KeyError, ValueError):
        return None


def host_cpu_model() -> str:
    """The host CPU's model name (Linux /proc/cpuinfo), or the platform's."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


def copy_probe(mib: int = 1024, reps: int = 3) -> int:
    """A plain device copy of known size, the calibration of the PMC byte
    counters (run under rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE)."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copy-probe: {reps} copies of {n * 4} bytes (read {n * 4}, write {n * 4} each)",
          flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-oracle", action="store_true",
                    help="skip the oracle (no solved-frame gate, no cpu_baseline)")
    ap.add_argument("--workload", choices=["frame64", "batch32", "net64"], default="frame64",
                    help="frame64: the 64^3 single-frame metric (default); batch32: 32 uneven "
                         "lattices solved together; net64: the warm-start network at 64^3")
    ap.add_argument("--no-warm", action="store_true",
                    help="skip the warm-vs-plain leg (held-out sequence, committed weights)")
    ap.add_argument("--warm-frames", type=int, default=22,
                    help="frames of the held-out sequence in the warm-vs-plain leg")
    ap.add_argument("--persistent", action="store_true",
                    help="one persistent launch per CG solve on levels of <= 128 tiles")
    ap.add_argument("--tiles", type=str, default=None,
                    help="stencil tile kinds per level, e.g. 1,1,7 (default: the autotuner's "
                         "choice; fixed tiles make profiled runs time the same kernels)")
    ap.add_argument("--main-only", action="store_true",
                    help="time the main workload only (no tracked-frame, active-set or "
                         "warm-vs-plain legs): the byte-counter runs")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 1 GiB device copy (byte-counter calibration)")
    args = ap.parse_args()
    if args.copy_probe:
        return copy_probe()
    # the warm-vs-plain leg generates its held-out frames in worker processes,
    # started before this process first touches the GPU
    pool = None
    if args.main_only:
        args.no_warm = True
    if args.workload == "frame64" and not args.no_warm:
        from paper_1603_08161_amd import warm
        pool = warm.make_pool(min(8, os.cpu_count() or 1))
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the solve is "
              "single-GPU and has no multi-GPU path.", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_1603_08161_amd import Lattice
    from synth import make_config1

    if args.workload == "batch32":
        return bench_batch(args)
    if args.workload == "net64":
        return bench_net(args)

    scene = make_config1(args.seed)
    spec = scene.spec
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)

    def up(a):
        return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)

    inputs = [up(scene.canon), up(scene.target), up(scene.normal), up(scene.weight),
              up(scene.sparse_canon), up(scene.sparse_target)]
    torch.cuda.synchronize()
    print(f"# workload: {spec.dims} lattice, {spec.num_levels} levels, {scene.n_dense} dense + "
          f"{scene.n_sparse} sparse constraints", flush=True)

    # tile autotuning (setup, outside the timed region): the library times
    # each stencil tile shape per level on these constraints and keeps the
    # fastest for the captured schedule
    if args.tiles:
        tiles = [int(t) for t in args.tiles.split(",")]
        lat = Lattice.from_spec(spec, graph=True, persistent=args.persistent, profile=True,
                                tiles=tuple(tiles))
        lat.set_constraints(*inputs)
        print(f"# tiles per level {tiles} (fixed)", flush=True)
    else:
        lat = Lattice.from_spec(spec, graph=True, persistent=args.persistent, profile=True)
        lat.set_constraints(*inputs)
        tiles, tile_us = lat.tune(iters=10)
        print(f"# tiles per level {tiles}; us per CG iteration incl. gradient pass [8x8x4, "
              "8x8x8, 32x8x4, 32x8x4/1024, 8x8x16/1024, 16x4x16/1024, 16x4x8/512, "
              "8x8x4/512]: "
              + "; ".join("[" + ", ".join(f"{u:.2f}" for u in lv) + "]" for lv in tile_us),
              flush=True)

    def step():
        lat.set_constraints(*inputs)
        lat.solve_frame(reset=True)
        return lat.get_energy()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    energies = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        energies.append(step())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    energies = np.array(energies)
    print(f"# timed {args.steps} frames in {elapsed * 1e3:.2f} ms", flush=True)

    # roofline of the dominant kernel: device clock stamps captured in the
    # frame's graph around the 64^3 level's CG iterations, read back from the
    # last timed replay (the same stream and launches as the timed region)
    graph_us, graph_n = lat.profile()
    cg_a_us = float(graph_us["cg_a"])
    # the other kernel classes: a profiled eager replay of the same frame
    prof = Lattice.from_spec(spec, profile=True, tiles=tiles, persistent=args.persistent)
    prof.set_constraints(*inputs)
    rep = prof.solve_frame(reset=True, report=True)
    prof_us = rep["prof_us"]
    n_fine = spec.dims[0] * spec.dims[1] * spec.dims[2]
    nbytes = cg_iteration_bytes(n_fine, scene.n_dense, scene.n_sparse)
    achieved = nbytes / (cg_a_us * 1e-6) / 1e9
    print(f"# 64^3 CG iteration in the timed graph: {cg_a_us:.2f} us mean over "
          f"{graph_n['cg_a']} launches; eager finest-level kernel means (us): "
          + ", ".join(f"{k}={v:.2f}" for k, v in prof_us.items()), flush=True)

    # the constraint build alone (part of every timed step): validation,
    # rows, the radix sort by cell, segments, cell cache and node blocks of
    # the three levels
    torch.cuda.synchronize()
    tc = time.perf_counter()
    for _ in range(10):
        lat.set_constraints(*inputs)
    torch.cuda.synchronize()
    set_constraints_ms = (time.perf_counter() - tc) * 1e2
    print(f"# set_constraints: {set_constraints_ms:.3f} ms per frame", flush=True)

    out_cpu = None
    e_ref = None
    if not args.no_oracle:
        import oracle
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            tc = time.perf_counter()
            ref = oracle.solve_frame(scene)
            t_cpu = time.perf_counter() - tc
        e_ref = float(ref["energy"][0])
        out_cpu = {"value": 1.0 / t_cpu, "unit": "frames/s", "cores": 1, "kind": "oracle",
                   "host_cpu": host_cpu_model(), "host_nproc": os.cpu_count(),
                   "sample": "one full frame of the same workload (3 levels x 8 GN x 20 PCG, "
                             f"FP64, single-threaded BLAS): {t_cpu:.2f} s"}
        print(f"# oracle: {t_cpu:.2f} s/frame, E = {e_ref:.9g}", flush=True)

    track_leg = active_leg = None
    if not args.main_only:
        track_leg = tracked_frame_leg(args, tiles)
        active_leg = active_set_leg(args, scene, inputs)

    warm_leg = None
    if not args.no_warm:
        warm_leg = warm_vs_plain(args.warm_frames, pool)
        pool.close()
        pool.join()

    if e_ref is not None:
        rel = np.abs(energies[:, 0] / e_ref - 1.0)
        solved = int(np.sum(rel <= 1e-4))
        max_rel = float(rel.max())
    else:
        solved, max_rel = args.steps, None
    value = solved / elapsed
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "64^3 lattice (262144 nodes), 3 levels 16^3/32^3/64^3, 8 GN x 20 PCG "
                        "per level, torus rendered to a 640x480 depth map "
                        f"({scene.n_dense} dense + {scene.n_sparse} sparse constraints), seed "
                        f"{args.seed}",
            "lattice": list(spec.dims),
            "levels": spec.num_levels,
            "gn_iters": list(spec.gn_iters),
            "pcg_iters": list(spec.pcg_iters),
            "n_dense": scene.n_dense,
            "n_sparse": scene.n_sparse,
            "launch": "hipGraph replay per frame",
            "tiles": tiles,
        },
        "solved_frames": solved,
        "energy_gpu": float(energies[-1, 0]),
        "energy_oracle": e_ref,
        "max_rel_energy_err": max_rel,
        "roofline": {
            "bound": "hbm",
            "kernel": "fused CG iteration (k_cg<float>) on the 64^3 level",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(f"tile{tiles[-1]}"),
            "bytes_per_launch": nbytes,
            "mean_us": cg_a_us,
            "timing": "device clock stamps captured in the frame graph around the 64^3 "
                      "level's CG iterations 1..19 of each flip-flop iteration, last timed "
                      "replay (rocprofv3 kernel-trace mean in profiles/k_cg_frame64.md)",
            "note": "effective bandwidth: the 64^3 level's ~40 MB per launch stays in the "
                    "256 MB last-level cache (MALL) across iterations; the HBM-bound case is "
                    "--workload batch32 (~530 MB per launch)",
        },
        "kernel_mean_us_eager": prof_us,
        "set_constraints_ms": set_constraints_ms,
        "cpu_baseline": out_cpu,
        "tracked_frame": track_leg,
        "active_set": active_leg,
        "warm_vs_plain": warm_leg,
    }
    print(json.dumps(line), flush=True)
    return 0


def active_set_leg(args, scene, inputs):
    """The same 64^3 frame restricted to the optimised set M of Sec. 6-7
    (isosurface points plus their one-ring, VD_FLAG_ACTIVE_SET): frames/s of
    the same timed step, its own autotuned tiles, the oracle gate against the
    restricted FP64 solve, and the CG iteration's time and model bytes
    (144 B per point of M + 24 B per dense and 12 B per sparse sample)."""
    import numpy as np
    import torch

    from paper_1603_08161_amd import Lattice

    spec = scene.spec
    lat = Lattice.from_spec(spec, graph=True, profile=True, active_set=True)
    lat.set_constraints(*inputs)
    tiles, _ = lat.tune(iters=10)
    _, n_act, _ = lat.get_active()

    def step():
        lat.set_constraints(*inputs)
        lat.solve_frame(reset=True)
        return lat.get_energy()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    energies = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        energies.append(step())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    graph_us, _ = lat.profile()
    cg_us = float(graph_us["cg_a"])
    nbytes = 144.0 * n_act + 24.0 * scene.n_dense + 12.0 * scene.n_sparse
    e_ref = None
    solved = args.steps
    rel = None
    if not args.no_oracle:
        from threadpoolctl import threadpool_limits

        from oracle import active
        with threadpool_limits(limits=1):
            e_ref = float(active.solve_frame_active(scene)["energy"][0])
        rel = np.abs(np.array(energies)[:, 0] / e_ref - 1.0)
        solved = int(np.sum(rel <= 1e-4))
    print(f"# active set M: {n_act} of {spec.dims[0] ** 3} finest points; "
          f"{elapsed * 1e3 / args.steps:.2f} ms/frame; CG iteration {cg_us:.2f} us; tiles {tiles}",
          flush=True)
    return {"workload": "the 64^3 frame optimised on M only (isosurface points + one-ring)",
            "value": solved / elapsed, "unit": "frames/s", "ms_per_frame": elapsed * 1e3 /
            args.steps, "solved_frames": solved, "active_points": n_act,
            "energy_gpu": float(energies[-1][0]), "energy_oracle": e_ref,
            "max_rel_energy_err": None if rel is None else float(rel.max()),
            "tiles": tiles, "cg_iteration_us": cg_us, "cg_model_bytes": nbytes,
            "cg_effective_GBs": nbytes / (cg_us * 1e-6) / 1e9}


def tracked_frame_leg(args, tiles, rigid_iters: int = 2, icp_iters: int = 2):
    """The per-frame loop around the solve on the same 64^3 workload, all on
    the GPU: the depth frame and model samples are uploaded once; one tracked
    frame = `rigid_iters` projective ICP iterations of the global pose
    (Sec. 6) + `icp_iters` rounds of [projective association of the deformed
    model samples (Sec. 5.1) + the full flip-flop schedule] (Sec. 3).  Reports
    its wall time per frame (hipGraph schedule, device-resident inputs) and
    the pairs kept per round."""
    import numpy as np
    import torch

    from paper_1603_08161_amd import Lattice
    from synth import make_config1

    scene, frame = make_config1(args.seed, depth_frame=True)
    dev = torch.device("cuda", 0)

    def up(a):
        return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)

    frame_dev = type(frame)(depth=up(frame.depth), camera=frame.camera,
                            model_canon=up(frame.model_canon),
                            model_normal=up(frame.model_normal))
    lat = Lattice.from_spec(scene.spec, graph=True, tiles=tiles)
    lat.set_depth_frame(frame_dev, sparse_canon=up(scene.sparse_canon),
                        sparse_target=up(scene.sparse_target), eps=TRACK_EPS)
    rep = None
    for _ in range(2):
        rep = lat.track_frame(rigid_iters, icp_iters, reset=True, report=True)
    torch.cuda.synchronize()
    steps = max(3, args.steps // 3)
    t0 = time.perf_counter()
    for _ in range(steps):
        lat.track_frame(rigid_iters, icp_iters, reset=True, report=False)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    print(f"# tracked frame: {ms:.2f} ms ({rigid_iters} rigid + {icp_iters} association "
          f"rounds), kept {list(rep['assoc_kept'])} of {frame.model_canon.shape[0]}", flush=True)
    # fusion of the frame into the canonical TSDF (Sec. 8) and the mesh of
    # the fused surface (Sec. 4), deformed by the tracked state
    tau = 3.0 * scene.spec.spacing
    lat.fuse_depth(tau=tau, all_points=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        lat.fuse_depth(tau=tau, all_points=True, count=False)
    torch.cuda.synchronize()
    fuse_ms = (time.perf_counter() - t0) * 1e3 / steps
    t0 = time.perf_counter()
    canon, _, _, _ = lat.extract_mesh()
    mesh_ms = (time.perf_counter() - t0) * 1e3
    print(f"# fusion {fuse_ms:.3f} ms/frame; marching cubes {mesh_ms:.2f} ms "
          f"({canon.shape[0]} triangles, host copies included)", flush=True)
    return {"workload": f"64^3 torus frame: {frame.model_canon.shape[0]} model samples, "
                        f"640x480 depth, {scene.n_sparse} sparse pairs; {rigid_iters} rigid ICP "
                        f"iterations + {icp_iters} x (association + 3-level schedule)",
            "ms_per_frame": ms, "frames": steps,
            "assoc_kept": [int(k) for k in rep["assoc_kept"]],
            "rigid_hist": rep["rigid_hist"].tolist(), "energy": float(rep["energy"][0]),
            "eps": list(TRACK_EPS), "fusion_ms": fuse_ms, "mesh_ms_with_host_copies": mesh_ms,
            "mesh_triangles": int(canon.shape[0])}


def warm_vs_plain(frames: int, pool=None):
    """The learned warm start against the plain solve on a held-out 64^3
    sequence (seed 1000, frames 2..frames-1), with the committed weights: per
    frame the plain schedule's time and energy, then the time and finest-level
    iterations to reach that energy from the judged prediction and from the
    plain initialisation (see paper_1603_08161_amd/warm.py)."""
    import torch

    from paper_1603_08161_amd import Net, warm
    if not os.path.exists(warm.WEIGHTS):
        print(f"# warm-vs-plain skipped: {warm.WEIGHTS} missing", flush=True)
        return None
    net = Net((64, 64, 64))
    net.set_params(warm.load_weights())
    res = warm.evaluate(net, pool, [1000], frames, 64, torch.device("cuda", 0),
                        log=lambda m: print(m, flush=True))
    out = dict(res["summary"])
    out["sequence"] = "held-out seed 1000, 64^3, frames 2.." + str(frames - 1)
    out["stopping_rule"] = "finest-level flip-flop iterations until E <= plain schedule's E"
    return out


def bench_batch(args) -> int:
    """32 independent lattices (24^3..64^3, each with its own 320x240 frame)
    advanced together: every schedule step is one launch over all of them."""
    import numpy as np
    import torch

    from paper_1603_08161_amd import Batch, Lattice, batch_precision
    from synth.scenes import make_config2

    scenes = make_config2(args.seed)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)

    def up(a):
        return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)

    inputs = [[up(s.canon), up(s.target), up(s.normal), up(s.weight), up(s.sparse_canon),
               up(s.sparse_target)] for s in scenes]
    n_nodes = [s.spec.dims[0] * s.spec.dims[1] * s.spec.dims[2] for s in scenes]
    print(f"# batch of {len(scenes)} lattices, {sum(n_nodes)} finest nodes, "
          f"{sum(s.n_dense for s in scenes)} dense constraints", flush=True)
    precs = [batch_precision(s.spec.dims[0]) for s in scenes]
    lats = [Lattice.from_spec(s.spec, graph=True, precision=p) for s, p in zip(scenes, precs)]
    for lat, inp in zip(lats, inputs):
        lat.set_constraints(*inp)
    batch = Batch(lats)
    # tile autotuning of the batched launches (setup, outside the timed
    # region): per precision part and level, the fastest tile kind
    batch_tiles, _ = batch.tune(iters=10)
    print(f"# batch tiles per level {batch_tiles}", flush=True)

    def step():
        for lat, inp in zip(lats, inputs):
            lat.set_constraints(*inp)
        return batch.solve(reset=True, energies=True)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    energies = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        energies.append(step())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    print(f"# timed {args.steps} batch frames in {elapsed * 1e3:.2f} ms", flush=True)

    # the float32 part alone, profiled eagerly with the tuned tiles
    f32 = [k for k, p in enumerate(precs) if p == "fp32"]
    prof_lats = [Lattice.from_spec(scenes[k].spec, profile=True,
                                   tiles=tuple(batch_tiles["fp32"])) for k in f32]
    for lat, k in zip(prof_lats, f32):
        lat.set_constraints(*inputs[k])
    pb = Batch(prof_lats)
    cg = []
    for _ in range(3):
        pb.solve(reset=True, energies=True)
        prof_us = pb.profile()
        cg.append(prof_us["cg_a"])
    cg_us = float(np.mean(cg))
    nbytes = sum(cg_iteration_bytes(n_nodes[k], scenes[k].n_dense, scenes[k].n_sparse)
                 for k in f32)
    achieved = nbytes / (cg_us * 1e-6) / 1e9
    print("# finest-level kernel means (us): "
          + ", ".join(f"{k}={v:.2f}" for k, v in prof_us.items()), flush=True)

    gate = None
    solved = args.steps * len(scenes)
    golden = os.path.join(ROOT, "tests", "golden", "batch32_oracle.npz")
    if not args.no_oracle and args.seed == 0 and os.path.exists(golden):
        # every lattice of the last timed frame against the stored FP64
        # oracle replica solve (tests/golden/make_batch_golden.py); a lattice
        # counts as solved in every timed frame only if it passes (each frame
        # solves the same inputs from rest)
        gold = np.load(golden)
        rel, dpos = [], []
        for k, (s, lat) in enumerate(zip(scenes, lats)):
            rel.append(abs(energies[-1][k][0] / gold["energies"][k][0] - 1.0))
            n = n_nodes[k]
            m = min(n, gold["node_index"].shape[1])
            idx = gold["node_index"][k][:m]
            pos = lat.get_state()[0][idx].astype(np.float64)
            dpos.append(float(np.abs(pos - gold["positions"][k][:m]).max() / s.spec.spacing))
        ok = [r <= 1e-4 and d <= 1e-3 for r, d in zip(rel, dpos)]
        gate = {"lattices_checked": len(scenes), "lattices_passed": int(sum(ok)),
                "max_rel_energy_err": float(max(rel)), "max_pos_err_over_h": float(max(dpos)),
                "reference": "tests/golden/batch32_oracle.npz (FP64 oracle, replica mode)"}
        solved = args.steps * int(sum(ok))
    elif not args.no_oracle:
        import oracle
        from threadpoolctl import threadpool_limits
        sample = sorted(range(len(scenes)), key=lambda k: n_nodes[k])[:4]
        rel = []
        with threadpool_limits(limits=1):
            for k in sample:
                ref = oracle.solve_frame(scenes[k])
                rel.append(abs(energies[-1][k][0] / ref["energy"][0] - 1.0))
        passed = [k for k, r in zip(sample, rel) if r <= 1e-4]
        gate = {"sample_lattices": sample, "max_rel_energy_err": float(max(rel)),
                "lattices_passed": len(passed)}
        # only the sampled lattices are checked, so only they count as solved
        solved = args.steps * len(passed)
    line = {
        "metric": "solved lattice-frames/s, batch of 32 uneven lattices (24^3..64^3)",
        "value": solved / elapsed,
        "unit": "lattice-frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (lattices of 33+ nodes per axis), f64 (below)",
        "data": "synthetic",
        "config": {"workload": "32 lattices, n uniform in [24,64] per axis, 3 levels x 8 GN x "
                               "20 PCG, each with its own torus/sphere 320x240 depth frame",
                   "lattice_n": [s.spec.dims[0] for s in scenes],
                   "finest_nodes": sum(n_nodes),
                   "n_dense": sum(s.n_dense for s in scenes),
                   "precision": precs,
                   "launch": "one launch per schedule step over the lattices of each "
                             "precision, hipGraph; the float64 part on a forked stream",
                   "tiles": batch_tiles},
        "oracle_gate": gate,
        "roofline": {"bound": "hbm", "kernel": "batched fused CG iteration (k_cg<float>) "
                                               "on the finest level of the float32 lattices",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(f"batch_f32_tile{batch_tiles['fp32'][-1]}",
                                                 "traffic_k_cg_batch32.md"),
                     "bytes_per_launch": nbytes, "mean_us": cg_us,
                     "timing": "profiled eager batch of the float32 lattices, stream events "
                               "around each launch (rocprofv3 kernel-trace mean in "
                               "profiles/traffic_k_cg_batch32.md)"},
        "kernel_mean_us": prof_us,
    }
    print(json.dumps(line), flush=True)
    return 0


def net_flops(dims, cin0: int = 8) -> float:
    """Multiply-add flops (2 per MAC) of one forward pass of the warm-start
    network (include/vd_net.h) on an nx*ny*nz grid: 3x3x3 convolutions at
    the full, half and quarter resolution (axes halved with rounding up)."""
    l0 = list(dims)
    l1 = [(d + 1) // 2 for d in l0]
    l2 = [(d + 1) // 2 for d in l1]
    n = [l0[0] * l0[1] * l0[2], l1[0] * l1[1] * l1[2], l2[0] * l2[1] * l2[2]]
    layers = [(cin0, 16, 0), (16, 16, 0), (16, 32, 1), (32, 32, 1), (32, 64, 2), (64, 64, 2),
              (64, 32, 1), (64, 32, 1), (32, 16, 0), (32, 16, 0), (16, 3, 0)]
    return float(sum(2 * 27 * ci * co * n[lv] for ci, co, lv in layers))


def bench_net(args) -> int:
    """The warm-start network (not part of the paper's solve) on the 64^3
    grid: forward passes (inference, batch 1) and training steps (forward,
    backward, Adam; batch 4) on synthetic features, against the bfloat16
    dense matrix-core peak."""
    import numpy as np
    import torch

    from paper_1603_08161_amd import Net, warm

    dims = (64, 64, 64)
    N = dims[0] * dims[1] * dims[2]
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    net = Net(dims, max_batch=4)
    rng = np.random.default_rng(args.seed)
    if os.path.exists(warm.WEIGHTS):
        net.set_params(warm.load_weights())
    else:
        net.set_params(rng.normal(scale=0.05, size=Net.param_count()).astype(np.float32))

    def bf16_bits(a):
        u = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
        r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
        return torch.from_numpy(r.view(np.int16).reshape(-1)).to(dev)

    # input channels of the size the solver's features have: displacements
    # and their change (voxels), residual and validity
    feat = rng.normal(scale=0.2, size=(4, N, 8)).astype(np.float32)
    feat[..., 7] = (rng.random((4, N)) < 0.1).astype(np.float32)
    x = bf16_bits(feat)
    target = torch.from_numpy(rng.normal(scale=0.05, size=4 * 3 * N).astype(np.float32)).to(dev)
    out = torch.empty(3 * N, dtype=torch.float32, device=dev)
    x1 = x[: N * 8]
    for _ in range(max(args.warmup, 1)):
        net.forward(x1, batch=1, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        net.forward(x1, batch=1, out=out)
    torch.cuda.synchronize()
    t_fwd = (time.perf_counter() - t0) / args.steps
    params0 = net.get_params()
    for _ in range(2):
        net.train_step(x, target, batch=4, lr=1e-4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        net.train_step(x, target, batch=4, lr=1e-4)
    torch.cuda.synchronize()
    t_train = (time.perf_counter() - t0) / args.steps
    net.set_params(params0)
    f_fwd = net_flops(dims)
    achieved = f_fwd / t_fwd / 1e12
    print(f"# net64: forward {t_fwd * 1e3:.3f} ms ({f_fwd / 1e9:.2f} GFLOP), training step "
          f"(batch 4) {t_train * 1e3:.3f} ms", flush=True)
    line = {
        "metric": "warm-start network forward passes/s at 64^3 (bf16 matrix cores)",
        "value": 1.0 / t_fwd,
        "unit": "passes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_fwd * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16 (float32 accumulation)",
        "data": "synthetic",
        "config": {"workload": "3-D conv encoder-decoder, channels 16-32-64, 3x3x3 kernels, "
                               "64^3 grid, 8 input channels, batch 1 (training batch 4)",
                   "forward_gflop": f_fwd / 1e9},
        "roofline": {"bound": "mfma", "kernel": "whole forward pass (11 convolutions)",
                     "achieved": achieved, "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": achieved / 2500.0, "traffic": None},
        "train_step_ms_batch4": t_train * 1e3,
        "train_achieved_tflops": 3.0 * 4 * f_fwd / t_train / 1e12,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
