"""Host-side checks of the C-ABI (no GPU needed): the library loads and
exports every function include/vd.h and include/vd_net.h declare, the ctypes structures have the
C layout (checked against a gcc-compiled probe of the header), and argument
validation that happens before any device work."""

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vd.h")
HEADERS = [HEADER, os.path.join(ROOT, "include", "vd_net.h"),
           os.path.join(ROOT, "include", "vd_track.h"), os.path.join(ROOT, "include", "vd_fusion.h")]


def _declared():
    text = "".join(open(h).read() for h in HEADERS)
    return sorted(set(re.findall(r"^\s*(?:int|int64_t|const char\*)\s+(vd_\w+)\s*\(",
                                 text, re.M)))


def test_library_exports_every_declared_symbol():
    import paper_1603_08161_amd as vd
    lib = ctypes.CDLL(vd.LIB_PATH)
    names = _declared()
    assert len(names) >= 28
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(vd.EXPORTED) == names


def test_struct_layout_matches_header(tmp_path):
    import paper_1603_08161_amd._lib as L
    src = tmp_path / "probe.c"
    src.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "vd.h"
int main(void) {
  printf("desc %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(vd_lattice_desc),
         offsetof(vd_lattice_desc, spacing), offsetof(vd_lattice_desc, num_levels),
         offsetof(vd_lattice_desc, pcg_iters), offsetof(vd_lattice_desc, w_dense),
         offsetof(vd_lattice_desc, precision), offsetof(vd_lattice_desc, flags),
         offsetof(vd_lattice_desc, tile));
  printf("cons %zu %zu %zu\n", sizeof(vd_constraints), offsetof(vd_constraints, n_sparse),
         offsetof(vd_constraints, mem));
  printf("rep %zu %zu %zu %zu\n", sizeof(vd_solve_report), offsetof(vd_solve_report, n_trace),
         offsetof(vd_solve_report, trace), offsetof(vd_solve_report, prof_n));
  printf("opts %zu %zu %zu %zu\n", sizeof(vd_solve_opts), offsetof(vd_solve_opts, init_delta),
         offsetof(vd_solve_opts, energy_target), offsetof(vd_solve_opts, max_gn));
  printf("rep2 %zu %zu %zu\n", offsetof(vd_solve_report, init_energy),
         offsetof(vd_solve_report, warm_used), offsetof(vd_solve_report, target_reached));
  return 0;
}
''')
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)],
                   check=True)
    out = dict((l.split()[0], [int(x) for x in l.split()[1:]])
               for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                       check=True).stdout.splitlines())
    D = L.LatticeDesc
    assert out["desc"] == [ctypes.sizeof(D), D.spacing.offset, D.num_levels.offset,
                           D.pcg_iters.offset, D.w_dense.offset, D.precision.offset,
                           D.flags.offset, D.tile.offset]
    Cs = L.Constraints
    assert out["cons"] == [ctypes.sizeof(Cs), Cs.n_sparse.offset, Cs.mem.offset]
    R = L.SolveReport
    assert out["rep"] == [ctypes.sizeof(R), R.n_trace.offset, R.trace.offset, R.prof_n.offset]
    O = L.SolveOpts
    assert out["opts"] == [ctypes.sizeof(O), O.init_delta.offset, O.energy_target.offset,
                           O.max_gn.offset]
    assert out["rep2"] == [R.init_energy.offset, R.warm_used.offset, R.target_reached.offset]


def test_create_rejects_bad_descriptors_without_a_gpu():
    """Descriptor validation runs before any HIP call."""
    import paper_1603_08161_amd as vd
    from paper_1603_08161_amd._lib import LatticeDesc
    lib = vd.lib()
    good = dict(dims=(8, 8, 8), spacing=1.0, origin=(0, 0, 0), num_levels=2)
    cases = [
        dict(good, dims=(1, 8, 8)),
        dict(good, spacing=0.0),
        dict(good, spacing=float("nan")),
        dict(good, num_levels=0),
        dict(good, num_levels=5),
        dict(good, dims=(3, 3, 3), num_levels=3),  # 3 -> 2 -> 1
        dict(good, origin=(0, float("inf"), 0)),
        dict(good, tile=9),
        dict(good, tile=-1),
    ]
    for c in cases:
        d = LatticeDesc()
        for k in range(3):
            d.dims[k] = c["dims"][k]
            d.origin[k] = c["origin"][k]
        d.spacing = c["spacing"]
        d.num_levels = c["num_levels"]
        d.tile[1] = c.get("tile", 0)
        d.w_dense, d.w_sparse, d.w_arap = 1.0, 10.0, 5.0
        h = ctypes.c_void_p()
        assert lib.vd_lattice_create(ctypes.byref(d), None, ctypes.byref(h)) == vd.VD_EINVAL, c
    d = LatticeDesc()
    for k in range(3):
        d.dims[k] = 8
    d.spacing, d.num_levels, d.w_dense, d.w_sparse, d.w_arap = 1.0, 1, 1.0, -1.0, 5.0
    h = ctypes.c_void_p()
    assert lib.vd_lattice_create(ctypes.byref(d), None, ctypes.byref(h)) == vd.VD_EINVAL
    assert lib.vd_lattice_destroy(None) == vd.VD_OK
    assert lib.vd_solve_frame(None, None, None) == vd.VD_EINVAL
    assert vd.strerror(vd.VD_ERANGE).startswith("a canonical sample")


def test_fit_rotations_argument_checks_without_a_gpu():
    import paper_1603_08161_amd as vd
    lib = vd.lib()
    assert lib.vd_debug_fit_rotations(None, None, None, None, -1, 0, 0, None) == vd.VD_EINVAL
    assert lib.vd_debug_fit_rotations(None, None, None, None, 0, 7, 0, None) == vd.VD_EINVAL
    assert lib.vd_debug_fit_rotations(None, None, None, None, 0, 0, 0, None) == vd.VD_OK


def test_net_param_count_and_create_checks_without_a_gpu():
    import paper_1603_08161_amd._lib as L
    from oracle import net as onet
    assert L.Net.param_count() == sum(co * ci * 27 + co for _, ci, co, _, _ in onet.LAYERS)
    h = ctypes.c_void_p()
    for dims in [(0, 4, 4), (4, -1, 4)]:
        rc = L.lib().vd_net_create(dims[0], dims[1], dims[2], 1, None, ctypes.byref(h))
        assert rc == L.VD_EINVAL
    assert L.lib().vd_net_create(4, 4, 4, 0, None, ctypes.byref(h)) == L.VD_EINVAL
