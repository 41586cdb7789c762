"""The library's host code (mesh topology, internal partition, overlapping
decompositions, factor storage tables, block least squares) built with
AddressSanitizer and UndefinedBehaviorSanitizer by g++ and run on chamber
meshes, no GPU involved: tests/native/host_sanitize.cpp checks the outputs'
consistency (CSR structure, partition of unity sum_i R_i^T D_i R_i = I,
local orderings, storage ranges) and the process must end without a
sanitizer report."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import mw_inputs as mi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1607_02573_amd", "csrc")
HOST_SOURCES = ["topology.cpp", "decomp.cpp", "hostcheck.cpp", "blockls.cpp"]


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("g++ or the ROCm headers missing")
    out = str(tmp_path_factory.mktemp("asan") / "host_sanitize")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
           os.path.join(ROOT, "tests", "native", "host_sanitize.cpp"),
           *[os.path.join(CSRC, s) for s in HOST_SOURCES], "-o", out, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stderr[-4000:]
    return out


def write_mesh(path, w):
    m = w.mesh
    with open(path, "wb") as f:
        np.array([m.xyz.shape[0], m.tet.shape[0], m.bface.shape[0], w.n_sub], dtype=np.int32).tofile(f)
        np.ascontiguousarray(m.xyz, dtype=np.float64).tofile(f)
        np.ascontiguousarray(m.tet, dtype=np.int32).tofile(f)
        np.ascontiguousarray(m.bface, dtype=np.int32).tofile(f)
        np.ascontiguousarray(m.btag, dtype=np.int32).tofile(f)
        np.ascontiguousarray(w.part, dtype=np.int32).tofile(f)


@pytest.mark.parametrize("freq,n_sub", [(0.15e9, 8), (0.25e9, 13)])
def test_host_code_under_sanitizers(driver, tmp_path, freq, n_sub):
    w = mi.configs.small_chamber(freq, n_per_ring=8, n_sub=n_sub)
    mesh = str(tmp_path / "mesh.bin")
    write_mesh(mesh, w)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([driver, mesh], capture_output=True, text=True, timeout=900, env=env)
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0 and r.stdout.strip() == "OK", (r.returncode, r.stderr[-4000:])
