"""CPU robustness: the oracle and the host side of the HIP library run under
AddressSanitizer and UndefinedBehaviorSanitizer (no GPU needed).

  * the oracle is rebuilt with g++ -fsanitize=address,undefined and driven
    through every entry point on small scenes (both traversals, both wrap
    modes, the analytic and finite-difference adjoints, the L1 loss, the
    baked-SH shading), with out-of-bounds triangle ids and culled vertices;
  * the HIP library is rebuilt with instrumented host code only
    (-Xarch_host before every sanitizer flag; the gfx950 code is unchanged)
    and the C-ABI tests, whose validation paths reject bad arguments before
    anything is enqueued, run against it.

Any sanitizer report aborts its process (-fno-sanitize-recover=all), so the
test checks the exit status and the absence of reports.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

ORACLE_DRIVER = r'''
import sys
sys.path.insert(0, sys.argv[1])
import numpy as np
import oracle as O
import scenes as S
sc = S.make_config(1, resolution=(40, 32), tex_res=16)
cam = sc.cameras[0]
vis = O.raster_layers(sc.layers, cam)
assert np.array_equal(vis, O.raster_layers(sc.layers, cam, mode="brute"))
for wrap in (0, 1):
    img = O.shade(sc.layers, sc.textures, cam, vis, wrap=wrap)
g = S.upstream_grad(1, cam).astype(np.float64)
tgt = np.random.default_rng(0).uniform(0, 1, (cam.height, cam.width, 4)).astype(np.float32)
for wrap in (0, 1):
    O.backward(sc.layers, sc.textures, cam, vis, grad_out=g, wrap=wrap)
    O.backward(sc.layers, sc.textures, cam, vis, target=tgt, wrap=wrap)
    O.backward(sc.layers, sc.textures, cam, vis, target=tgt, wrap=wrap, loss="l1")
want = O.backward(sc.layers, sc.textures, cam, vis, grad_out=g)
ent = np.array([[0, 3, 4, 1], [2, 7, 8, 3]], np.int32)
O.finite_diff(sc.layers, sc.textures, cam, vis, ent, h=1e-3, grad_out=g)
O.coverage(sc.layers[0], cam)
O.project(sc.layers[0], cam)
sh = [S.sh_texture(70, l, 16, 12, degree=3, opaque=(l == 2)) for l in range(3)]
O.shade_sh(sc.layers, sh, cam, vis, degree=3)
# culled vertices, a zero-area triangle and out-of-range ids
xyz = np.array([[-0.5, -0.5, 1.0], [0.5, -0.5, 1.0], [0.0, 0.5, 1.0], [0.0, 0.0, 0.001],
                [np.nan, 0.0, 1.0]], np.float32)
tri = np.array([[0, 1, 2], [0, 1, 3], [0, 1, 4], [0, 0, 1], [0, 1, 77], [-5, 1, 2]], np.int32)
mesh = S.Mesh(xyz, np.full((5, 2), 0.5, np.float32), tri)
c2 = S.Camera(16, 12, 8.0, 8.0, 8.0, 6.0, np.eye(3), np.zeros(3))
v2 = O.raster_layers([mesh], c2)
O.shade([mesh], [S.constant_texture(4, 4, [1, 0.5, 0.25, 1])], c2, v2)
print("oracle clean")
'''


def _run(cmd, env, timeout):
    r = subprocess.run(cmd, env=env, capture_output=True, text=True, timeout=timeout)
    out = r.stdout + r.stderr
    return r.returncode, out


def test_oracle_under_asan_and_ubsan(tmp_path):
    lib = tmp_path / "libvs_oracle_san.so"
    subprocess.check_call(["g++", "-O1", "-g", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                           "-shared", "-fPIC", os.path.join(ROOT, "oracle", "vs_oracle.cpp"), "-o", str(lib)])
    asan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", VS_ORACLE_LIB=str(lib))
    code, out = _run([sys.executable, "-c", ORACLE_DRIVER, ROOT], env, 600)
    assert code == 0 and "oracle clean" in out, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]


def _clang_asan_runtime():
    import glob
    hits = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


@pytest.mark.slow
def test_host_library_under_asan_and_ubsan(tmp_path):
    from paper_2409_02482_amd import build as hb
    rt = _clang_asan_runtime()
    if rt is None:
        pytest.skip("no clang ASan runtime in this image")
    lib = tmp_path / "libvs_hostsan.so"
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    cmd = [hb.HIPCC, *hb.FLAGS, *san, *hb.sources(), "-o", str(lib)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    syms = subprocess.run(["nm", "-D", str(lib)], capture_output=True, text=True).stdout
    assert "__asan_" in syms and "__ubsan_" in syms, "host code is not instrumented"
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", VS_LIB=str(lib))
    code, out = _run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                      os.path.join(ROOT, "tests", "test_abi.py")], env, 900)
    assert code == 0 and " passed" in out, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
