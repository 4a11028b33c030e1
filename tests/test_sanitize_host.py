"""The host C++ mesh set-up and the C oracle built with AddressSanitizer and
UndefinedBehaviorSanitizer (g++/gcc, CPU only) and run on small workloads:
the dam-break canal, a river reach with inflow and a fixed outlet stage, a
two-triangle mesh, each mesh also given as an edge list, and broken meshes
that must be refused. A sanitizer finding aborts the test program (no recovery)
and fails the test."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-g", "-O1", "-fno-omit-frame-pointer", "-fopenmp",
       "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def _build(tmp):
    gxx, gcc = shutil.which("g++"), shutil.which("gcc")
    if not gxx or not gcc:
        pytest.skip("no host compiler")
    csrc = os.path.join(ROOT, "paper_2010_14416_amd", "csrc")
    mesh = os.path.join(tmp, "mesh_asan")
    subprocess.check_call([gxx, "-std=c++17", *SAN, f"-I{csrc}",
                           os.path.join(ROOT, "tests", "sanitize",
                                        "mesh_driver.cpp"),
                           os.path.join(csrc, "swe_mesh.cpp"), "-o", mesh])
    ora = os.path.join(tmp, "oracle_asan")
    subprocess.check_call([gcc, "-std=c99", *SAN, "-ffp-contract=off",
                           os.path.join(ROOT, "tests", "sanitize",
                                        "oracle_driver.c"),
                           os.path.join(ROOT, "oracle", "swe_oracle.c"),
                           "-lm", "-o", ora])
    return mesh, ora


def _write(case, path):
    en, ec, et = W.edge_list(case, seed=3)
    with open(path, "wb") as f:
        np.array([case.xy.shape[0]], np.int64).tofile(f)
        np.ascontiguousarray(case.xy, np.float64).tofile(f)
        np.array([case.n_cells], np.int64).tofile(f)
        np.ascontiguousarray(case.tri, np.int32).tofile(f)
        bnd = np.ascontiguousarray(case.bnd, np.int32).reshape(-1, 2)
        np.array([bnd.shape[0]], np.int64).tofile(f)
        bnd.tofile(f)
        np.ascontiguousarray(case.bnd_tag, np.int32).tofile(f)
        np.array([len(et)], np.int64).tofile(f)
        np.ascontiguousarray(en, np.int32).tofile(f)
        np.ascontiguousarray(ec, np.int32).tofile(f)
        np.ascontiguousarray(et, np.int32).tofile(f)
        (case.h > case.h_dry).astype(np.uint8).tofile(f)
        for a in (case.z, case.manning, case.h, case.hu, case.hv):
            np.ascontiguousarray(a, np.float64).tofile(f)
        np.array([len(case.bc)], np.int32).tofile(f)
        for tag, (kind, value) in case.bc.items():
            np.array([tag, kind], np.int32).tofile(f)
            np.array([value], np.float64).tofile(f)


def _cases():
    xy = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], float)
    tri = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    tiny = W.Case(name="two-triangles", xy=xy, tri=tri,
                  bnd=np.zeros((0, 2), np.int32),
                  bnd_tag=np.zeros(0, np.int32), bc={},
                  z=np.array([0.0, 0.1]), manning=np.array([0.02, 0.03]),
                  h=np.array([1.0, 0.2]), hu=np.array([0.1, 0.0]),
                  hv=np.array([0.0, -0.05]))
    return [W.dam_break_canal(), W.river(n_target=6_000, workers=1), tiny]


@pytest.mark.slow
def test_mesh_setup_and_oracle_under_sanitizers(tmp_path):
    mesh, ora = _build(str(tmp_path))
    env = dict(os.environ, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    for k, case in enumerate(_cases()):
        path = str(tmp_path / f"case{k}.bin")
        _write(case, path)
        for exe in (mesh, ora):
            r = subprocess.run([exe, path], capture_output=True, text=True,
                               env=env, timeout=600)
            assert r.returncode == 0, (case.name, exe, r.stdout[-2000:],
                                       r.stderr[-4000:])
            assert "runtime error" not in r.stderr, r.stderr[-4000:]
