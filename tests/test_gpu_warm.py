"""The trained warm start (committed weights) on a held-out 64^3 sequence,
against the method without it.

Per frame, from the previous frame's plain solution: the plain schedule sets
the energy to reach; the judged network prediction and the plain
initialisation then run finest-level iterations until they reach it.  The
test prints what the network gains (initial energy, iterations, time, the
warm start's factor over the plain initialisation under the same stopping
rule, prediction error against predicting no change) and checks what the
design guarantees: the judge never starts above the plain initialisation,
the warm path reaches the target whenever the plain initialisation does, and
a rejected prediction leaves exactly the plain-initialisation run (same
iterations, same final energy bits).  Whether the network gains is measured
and reported, not asserted: it is a property of the trained weights."""

import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_trained_warm_start_on_a_held_out_sequence():
    import torch

    from paper_1603_08161_amd import Net, warm
    assert os.path.exists(warm.WEIGHTS), "trained weights missing"
    net = Net((64, 64, 64))
    net.set_params(warm.load_weights())
    res = warm.evaluate(net, None, [1000], 10, 64, torch.device("cuda", 0), max_gn=16,
                        log=print)
    s = res["summary"]
    print("summary", s)
    for r in res["frames"]:
        start = r["e_init_warm"] if r["warm_used"] else r["e_init_plain"]
        assert start <= r["e_init_plain"]
        assert r["reached_warm"] >= r["reached_plain"]
        assert np.isfinite(r["pred_mse"])
        if not r["warm_used"]:
            assert r["gn_warm"] == r["gn_plain_target"]
            assert r["e_warm"] == r["e_plain_target"]
        # the exact step along the prediction never starts above the plain
        # initialisation and reaches the target whenever that does
        start = r["e_init_step"] if r["step_used"] else r["e_init_plain"]
        assert start <= r["e_init_plain"]
        assert r["reached_step"] >= r["reached_plain"]
    print(f"warm-start factor (plain-init time / warm time, same stopping rule): "
          f"{s['warm_start_factor']:.3f}; iterations {s['gn_plain_init_mean']:.2f} plain-init "
          f"vs {s['gn_warm_mean']:.2f} warm")
    print(f"exact step along the prediction: factor {s['warm_step_factor']:.3f}, used on "
          f"{s['step_used_frac']:.2f} of the frames, initial energy ratio "
          f"{s['step_init_energy_ratio_mean']:.4f}, iterations {s['gn_step_mean']:.2f}")
    assert np.isfinite(s["warm_start_factor"]) and s["warm_start_factor"] > 0
