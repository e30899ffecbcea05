"""The oracle built with AddressSanitizer (host code only) and driven through
its whole interface in a child process: tracking with and without a mesh
tally, ray mode, traces, births, find_cell and distance_to_surface, and the
work meter, on small cases of every workload shape."""

import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_oracle_under_address_sanitizer(tmp_path):
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("no gcc")
    rt = subprocess.run([cc, "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not rt or not os.path.isabs(rt) or not os.path.exists(rt):
        pytest.skip("no AddressSanitizer runtime")
    lib = str(tmp_path / "liboracle_asan.so")
    subprocess.run([cc, "-O1", "-g", "-fsanitize=address", "-fno-omit-frame-pointer", "-shared", "-fPIC", "-o", lib,
                    os.path.join(ROOT, "oracle", "oracle.c"), "-lm", "-lpthread"], check=True)
    code = r"""
import sys
sys.path.insert(0, %r)
import oracle
oracle.LIB = %r
print("loaded", oracle.lib()._name)
from paper_2406_13849_amd import synth
for name in ("cfg1", "cfg2", "cfg4", "sphere", "hex_pin_box", "nested_box"):
    fg = synth.make_config(int(name[3:])) if name.startswith("cfg") else getattr(synth, name)()
    O = oracle.OracleGeometry(fg)
    p = oracle.TrackParams(seed=5, n_particles=300, geometry_id=3, record_first_k=20, record_cap=16)
    oracle.track(O, p, n_threads=3)
    oracle.track(O, p, n_threads=2, mesh=(fg.domain_lo - 0.5, fg.domain_hi * 0.7, (5, 3, 4)))
    oracle.track(O, oracle.TrackParams(seed=5, n_particles=64, source=1, ray_n1=8), n_threads=1,
                 mesh=(fg.domain_lo, fg.domain_hi, (2, 9, 1)))
    oracle.trace_particle(O, p, 3)
    pos, d, tau, inst = oracle.sample_births(O, p)
    O.find_cell(pos)
    O.distance_to_surface(pos, d)
    oracle.count_work(O, oracle.TrackParams(seed=5, n_particles=50, geometry_id=3))
print("asan clean")
""" % (ROOT, lib)
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0 and "asan clean" in r.stdout, (r.stdout[-2000:] + r.stderr[-4000:])
    assert ("loaded " + lib) in r.stdout
