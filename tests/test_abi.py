"""The C ABI library: it loads without a GPU, exports every entry point the
header declares, its structs match the header's layout, its host-side calls
agree with the oracle's tables, and argument errors are reported, all
without touching a device."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from oracle import oracle as orc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


def _lbm():
    from paper_2012_06144_amd import lbm
    return lbm


def _declared_functions(path):
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lbm = _lbm()
    declared = _declared_functions(HEADER)
    assert len(declared) >= 15
    out = subprocess.run(["nm", "-D", "--defined-only", lbm.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (lbm_[a-z_0-9]+)$", out, flags=re.M))
    missing = [f for f in declared if f not in exported]
    assert not missing, missing
    assert sorted(lbm.EXPORTS) == declared


def test_surrogate_library_exports_every_declared_symbol():
    lbm = _lbm()
    from paper_2012_06144_amd import sg
    declared = sorted(set(re.findall(r"\b(sg_[a-z_0-9]+)\s*\(",
                                     re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "sg.h")).read(),
                                            flags=re.S))))
    assert len(declared) >= 15
    out = subprocess.run(["nm", "-D", "--defined-only", lbm.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (sg_[a-z_0-9]+)$", out, flags=re.M))
    assert not [f for f in declared if f not in exported]
    assert sorted(sg.EXPORTS) == declared


def test_struct_layout_matches_header(tmp_path):
    """Compile a probe against include/lbm.h with gcc and compare sizes and
    offsets with the ctypes mirrors used by the binding."""
    lbm = _lbm()
    src = tmp_path / "probe.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "lbm.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(lbm_params), offsetof(lbm_params, body_accel),
         offsetof(lbm_params, storage), offsetof(lbm_params, density_literal), sizeof(lbm_stats),
         offsetof(lbm_params, lattice_phase), offsetof(lbm_params, phase_mrt));
  printf("%zu %zu\\n", offsetof(lbm_stats, centroid), offsetof(lbm_stats, max_speed));
  return 0;
}
""")
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                           check=True).stdout.split()]
    P, S = lbm.LbmParams, lbm.LbmStats
    assert vals[:7] == [C.sizeof(P), P.body_accel.offset, P.storage.offset, P.density_literal.offset,
                        C.sizeof(S), P.lattice_phase.offset, P.phase_mrt.offset]
    assert vals[7:] == [S.centroid.offset, S.max_speed.offset]


@pytest.mark.parametrize("q", [15, 19, 27])
def test_velocity_set_matches_oracle(q):
    lbm = _lbm()
    e, w = lbm.lbm_velocity_set(q)
    eo, wo = orc.velocity_set(q)
    assert np.array_equal(e, eo)
    assert np.array_equal(w, wo)


def test_velocity_set_rejects_other_q():
    lbm = _lbm()
    for q in (9, 21, 0):
        with pytest.raises(lbm.LbmError):
            lbm.lbm_velocity_set(q)


@pytest.mark.parametrize("bad", [
    dict(mobility=0.0), dict(tau_L=0.0), dict(tau_H=-1.0), dict(xi=0.0), dict(phi_H=0.0),
    dict(rho_L=0.0), dict(storage=7), dict(lattice_phase=19, lattice_hydro=27),
    dict(lattice_phase=21), dict(lattice_hydro=21), dict(lattice_phase=19, lattice_hydro=19, storage="f16s"),
])
def test_workspace_bytes_rejects_bad_parameters(bad):
    lbm = _lbm()
    kw = dict(nx=8, ny=8, nz=8)
    kw.update(bad)
    p = lbm.make_params(**kw)
    with pytest.raises(lbm.LbmError):
        lbm.lbm_workspace_bytes(p)


def test_workspace_bytes_grid_limits():
    lbm = _lbm()
    with pytest.raises(lbm.LbmError):
        lbm.lbm_workspace_bytes(lbm.make_params(0, 8, 8))
    with pytest.raises(lbm.LbmError):
        lbm.lbm_workspace_bytes(lbm.make_params(8, 2, 8, walls_y=True))
    with pytest.raises(lbm.LbmError, match="2\\^31"):
        lbm.lbm_workspace_bytes(lbm.make_params(2048, 2048, 1024))
    # 512^3, FP32 storage: two-grid PDFs (84 values) + 2 phi + u = 356 B per cell
    n = lbm.lbm_workspace_bytes(lbm.make_params(512, 512, 512, walls_y=True, storage="f32"))
    assert 355 * 512 ** 3 < n < 358 * 512 ** 3
    n = lbm.lbm_workspace_bytes(lbm.make_params(512, 512, 512, walls_y=True, storage="f16s"))
    assert 187 * 512 ** 3 < n < 190 * 512 ** 3   # 84 half PDFs + 2 phi + u in FP32


def test_create_validates_without_device_access():
    """lbm_create checks size and alignment before touching memory; calls
    out of order report LBM_ESTATE / LBM_EARG (no device work is issued)."""
    lbm = _lbm()
    p = lbm.make_params(16, 16, 16)
    need = lbm.lbm_workspace_bytes(p)
    fake = 1 << 40  # never dereferenced by the checks below
    with pytest.raises(lbm.LbmError, match="workspace has"):
        lbm.lbm_create(p, fake, need - 1, 0)
    with pytest.raises(lbm.LbmError, match="aligned"):
        lbm.lbm_create(p, fake + 8, need, 0)
    ctx = lbm.lbm_create(p, fake, need, 0)
    try:
        with pytest.raises(lbm.LbmError, match="not initialised"):
            lbm.lbm_step(ctx, 1)
        with pytest.raises(lbm.LbmError, match="not initialised"):
            lbm.lbm_reduce_mass(ctx)
        assert lbm.lbm_steps_done(ctx) == 0
    finally:
        lbm.lbm_destroy(ctx)


def test_one_hip_runtime_per_process():
    """Importing the package before torch must still leave one HIP runtime in
    the process (torch's), or the library and torch would each bring up
    their own and the library would see no device."""
    import subprocess
    import sys
    code = ("import paper_2012_06144_amd.surrogate, torch\n"
            "m = open('/proc/self/maps').read().splitlines()\n"
            "print(len(set(l.split()[-1] for l in m if 'libamdhip64' in l)))\n")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300,
                         cwd=os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    assert out.returncode == 0, out.stderr[-2000:]
    assert out.stdout.strip().splitlines()[-1] == "1"
