"""CPU check of the library's rotation fit (vd_device.h compiled for the
host with hipcc --cuda-host-only) against the oracle's SVD Procrustes:
random covariances, reflections (det < 0), near-identity, exactly rank-1
(degenerate: previous rotation kept), and warm starts from arbitrary previous
rotations (the fit must not depend on the starting point)."""

import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle.procrustes import fit_rotations
from synth import random_rotation

from helpers import edge_fit_cases, rotation_angle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "fit_host.cpp")

pytestmark = pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists(
    "/opt/rocm/bin/hipcc"), reason="hipcc not available")


@pytest.fixture(scope="module")
def fit_exe(tmp_path_factory):
    exe = tmp_path_factory.mktemp("fit") / "fit_host"
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    subprocess.run([hipcc, "--cuda-host-only", "-O2", "-std=c++17", SRC, "-o", str(exe)],
                   check=True, capture_output=True)
    return str(exe)


def _run(exe, M, Rp, prec):
    lines = [f"{M.shape[0]} {prec}"]
    for m, r in zip(M.reshape(-1, 9), Rp.reshape(-1, 9)):
        lines.append(" ".join(repr(float(v)) for v in np.concatenate([m, r])))
    out = subprocess.run([exe], input="\n".join(lines), capture_output=True, text=True,
                         check=True).stdout.split("\n")
    vals = np.array([[float(v) for v in l.split()] for l in out if l.strip()])
    return vals[:, 1:].reshape(-1, 3, 3), vals[:, 0].astype(int)


def _cases(seed, n=400):
    rng = np.random.default_rng(seed)
    M = rng.normal(size=(n, 3, 3))
    M[::3, :, 0] *= -1.0
    M[1::9] = np.eye(3) + 1e-3 * rng.normal(size=M[1::9].shape)
    a = rng.integers(1, 4, size=(n, 3)) * rng.choice([-1, 1], size=(n, 3))
    b = rng.integers(1, 4, size=(n, 3)) * rng.choice([-1, 1], size=(n, 3))
    M[4::50] = np.einsum("ka,kb->kab", a, b)[: M[4::50].shape[0]]
    M[7::50] = 0.0
    Rp = np.stack([random_rotation(rng) for _ in range(n)])
    return M.astype(np.float32).astype(np.float64), Rp.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("prec,tol", [(0, 1e-5), (1, 1e-10)])
def test_fit_matches_oracle(fit_exe, prec, tol):
    M, Rp = _cases(1)
    R_ref, deg = fit_rotations(M, Rp)
    R, code = _run(fit_exe, M, Rp, prec)
    np.testing.assert_array_equal(code == 2, deg)
    np.testing.assert_allclose(R[deg], Rp[deg], atol=1e-7)
    ang = rotation_angle(R[~deg], R_ref[~deg])
    assert ang.max() < tol, ang.max()


def test_fit_independent_of_warm_start(fit_exe):
    M, _ = _cases(2, n=200)
    deg = fit_rotations(M)[1]
    rng = np.random.default_rng(3)
    R1, _ = _run(fit_exe, M, np.broadcast_to(np.eye(3), M.shape).copy(), 1)
    R2, _ = _run(fit_exe, M, np.stack([random_rotation(rng) for _ in range(M.shape[0])]), 1)
    assert rotation_angle(R1[~deg], R2[~deg]).max() < 1e-10


@pytest.mark.parametrize("prec,tol", [(0, 1e-5), (1, 1e-10)])
def test_fit_edge_cases(fit_exe, prec, tol):
    """Nearly diagonal (rotation angles down to 1e-33) and 1e-15 / 1e15-scaled
    cross-covariances: the host build of the fit matches the oracle's SVD."""
    M, Rp = edge_fit_cases(12)
    R_ref, deg = fit_rotations(M, Rp)
    assert not deg.any()
    R, code = _run(fit_exe, M, Rp, prec)
    assert not (code == 2).any()
    ang = rotation_angle(R, R_ref)
    assert ang.max() < tol, ang.max()
