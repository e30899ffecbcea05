"""The C ABI library: it loads, exports every entry point include/gt.h
declares, and rejects invalid geometries and arguments with the documented
codes before touching the GPU (no compute calls here)."""

import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2406_13849_amd import gt, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "gt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gt_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = gt.lib()
    names = _declared()
    assert "gt_track" in names and "gt_geometry_create" in names
    for n in names:
        assert hasattr(L, n), n


def _create(g):
    keep = []
    f = gt.flat_struct(g, keep)
    h = C.c_void_p()
    rc = gt.lib().gt_geometry_create(C.byref(f), C.byref(h))
    return rc, gt.lib().gt_last_error().decode()


def _cfg1():
    return synth.make_config(1)


@pytest.mark.parametrize("mutate,code,needle", [
    (lambda g: g.hs.__setitem__(0, 999), gt.GT_EGEOM, "names no surface"),
    (lambda g: g.hs.__setitem__(0, 0), gt.GT_EGEOM, "names no surface"),
    (lambda g: g.cell_fill.__setitem__(0, -99), gt.GT_EGEOM, "daughter universe"),
    (lambda g: g.cell_fill.__setitem__(10, 50), gt.GT_EGEOM, "material"),
    (lambda g: g.sigma_t.__setitem__(0, 0.0), gt.GT_EGEOM, "sigma_t"),
    (lambda g: g.surf_type.__setitem__(0, 9), gt.GT_EGEOM, "unknown type"),
    (lambda g: g.cell_fill.__setitem__(9, -2), gt.GT_EGEOM, "cycle"),
    (lambda g: g.domain_hi.__setitem__(0, -5.0), gt.GT_EGEOM, "domain"),
    (lambda g: g.lattice_hint.__setitem__((0, 1), 4), gt.GT_EGEOM, "lattice hint"),
])
def test_invalid_geometry_rejected(mutate, code, needle):
    g = _cfg1()
    for a in ("hs", "cell_fill", "sigma_t", "surf_type", "domain_hi", "lattice_hint"):
        setattr(g, a, getattr(g, a).copy())
    mutate(g)
    rc, msg = _create(g)
    assert rc == code, (rc, msg)
    assert needle in msg


def test_surface_shared_between_universes_rejected():
    g = _cfg1()
    g.hs = g.hs.copy()
    # the pin universe's first cell uses the root's first lattice plane
    pin_cell = int(g.univ_cell_off[1])
    g.hs[g.cell_hs_off[pin_cell]] = 1
    rc, msg = _create(g)
    assert rc == gt.GT_EGEOM and "used by universes" in msg


def test_root_cell_outside_domain_rejected():
    g = _cfg1()
    g.domain_hi = g.domain_hi.copy()
    g.domain_hi[2] = 1.0   # root cells reach z = 1.875
    rc, msg = _create(g)
    assert rc == gt.GT_EGEOM and "domain box" in msg


def test_null_arguments():
    L = gt.lib()
    assert L.gt_geometry_create(None, None) == gt.GT_EINVAL
    assert L.gt_track(None, None, None, None) == gt.GT_EINVAL
    assert L.gt_find_cell(None, None, 1, None, None, 0, None) == gt.GT_EINVAL
    assert L.gt_fp64_check(None, None, 5, None, None, None, None) == gt.GT_EINVAL


def test_binding_struct_layouts_match_the_header(tmp_path):
    """The ctypes structures of the binding have the header's sizes and
    field offsets (a C program compiled against include/gt.h prints them)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"gt_track_params": gt._Params, "gt_track_out": gt._Out, "gt_batch_item": gt._BatchItem,
               "gt_tuning": gt._Tuning, "gt_launch_info": gt._LaunchInfo, "gt_flat_geometry": gt._Flat,
               "gt_mesh": gt._Mesh}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "gt.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (name, name))
        for f, _ in cls._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (name, f, name, f))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for ln in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines():
        k, v = ln.rsplit(" ", 1)
        got[k] = int(v)
    for name, cls in structs.items():
        assert got["%s size" % name] == C.sizeof(cls), name
        for f, _ in cls._fields_:
            assert got["%s %s" % (name, f)] == getattr(cls, f).offset, (name, f)


def test_mesh_workspace_bytes_follows_the_replica_rule():
    """A mesh workspace holds four 64-bit limb counters per bin in each
    replica: one replica per XCD (eight) while those take at most 64 MB,
    a single one above that; 0 for no bins or more than 2^31."""
    L = gt.lib()
    L.gt_mesh_workspace_bytes.argtypes = [C.c_uint64]
    L.gt_mesh_workspace_bytes.restype = C.c_uint64
    assert L.gt_mesh_workspace_bytes(0) == 0
    assert L.gt_mesh_workspace_bytes((1 << 31) + 1) == 0
    for bins in (1, 1000, 262_144):
        assert L.gt_mesh_workspace_bytes(bins) == 8 * 32 * bins
    for bins in (262_145, 119 * 119 * 30, 1 << 31):
        assert L.gt_mesh_workspace_bytes(bins) == 32 * bins
