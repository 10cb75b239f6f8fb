"""The library's host code under the compiler's sanitizers (CPU only).

tests/sanitize_host.cpp drives the host sources -- the threaded list
builder (polygons in parallel, one large polygon split over threads), the
MBR join, list files, list validation -- built with g++ twice:
AddressSanitizer + UndefinedBehaviorSanitizer, and ThreadSanitizer.  A
sanitizer report, or a failed check, fails the test.  The workload: 400
polygons of the tiny distribution and one 4,000-vertex star polygon, on a
grid of order 13.
"""

import os
import subprocess

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2307_01716_amd", "csrc")
SOURCES = [os.path.join(ROOT, "tests", "sanitize_host.cpp")] + [
    os.path.join(CSRC, f) for f in ("build.cpp", "lists.cpp", "lists_io.cpp")]
FLAGS = {
    "address": ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"],
    "thread": ["-fsanitize=thread"],
}


@pytest.fixture(scope="module")
def workload(tmp_path_factory):
    d = tmp_path_factory.mktemp("sanitize")
    R, _, _ = synth.configs.tiny(n=400)
    rng = np.random.default_rng(77)
    big = synth.star_polygons(rng, np.array([[0.5, 0.5]]), np.array([0.15]), np.array([4000]), a=0.3)
    P = synth.PolygonSet.concat(big, R)
    g = synth.grid_covering([P], 13)
    path = d / "polys.bin"
    with open(path, "wb") as f:
        np.array([len(P), len(P.xy)], np.uint64).tofile(f)
        np.ascontiguousarray(P.voff, np.uint64).tofile(f)
        np.ascontiguousarray(P.xy, np.float64).tofile(f)
        np.array([g.x0, g.y0, g.side], np.float64).tofile(f)
        np.array([g.order], np.uint64).tofile(f)
    return d, path


@pytest.mark.parametrize("kind", list(FLAGS))
def test_host_code_under_sanitizer(workload, kind):
    d, path = workload
    exe = d / f"sanitize_{kind}"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", *FLAGS[kind], "-pthread",
           "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           "-I", "/opt/rocm/include", *SOURCES, "-L/opt/rocm/lib", "-lamdhip64",
           "-Wl,-rpath,/opt/rocm/lib", "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True)
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["TSAN_OPTIONS"] = "halt_on_error=1"
    run = subprocess.run([str(exe), str(path), str(d)], capture_output=True, text=True, env=env,
                         timeout=600)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "Sanitizer" not in run.stderr, run.stderr
    assert "sanitize_host ok" in run.stdout
