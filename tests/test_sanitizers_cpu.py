"""AddressSanitizer and UndefinedBehaviorSanitizer runs of the host code (CPU).

* the FP64 oracle (oracle/oracle.c, built with gcc): plain renders with and
  without its BVH, a coated scene, a radiance-cache render with training rows,
  a window render and the path probe (tests/sanitize/oracle_driver.c);
* the library's host code (api.cpp, bvh_build.cpp, built for the host with the
  sanitizers; the device code is linked uninstrumented and never launched):
  scene validation on good and damaged scenes, the grid and binned-SAH BVH
  builder over four grids and three leaf sizes, launch-setting checks and the
  tuning results file (tests/sanitize/host_driver.cpp).

Each runs on the tiny room, its coated variant and the point-light-behind-
panes fixture; a sanitizer report or a failed check fails the test.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import scenegen as sg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_1912_06474_amd", "csrc")
OBJ = os.path.join(ROOT, "paper_1912_06474_amd", "_build")
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")

SCENES = {
    "tiny": lambda: sg.tiny_room(0, 16),
    "coated": lambda: sg.tiny_room(0, 16, coating_state=0.6),
    "point_panes": lambda: sg.point_light_panes(16, seed=3),
}


def _write_scene(sc, d):
    os.makedirs(d, exist_ok=True)
    arrays = dict(verts=np.float32, tris=np.int32, tri_mat=np.int32, lambda_nm=np.float32, lambda_w=np.float64,
                  cmf=np.float64, mat_type=np.int32, mat_rho=np.float32, mat_n=np.float32, mat_k=np.float32,
                  mat_thick=np.float32, mat_le=np.float32, light_p0=np.float32, light_e1=np.float32,
                  light_e2=np.float32)
    lm = 0
    if "mat_n_layers" in sc:
        arrays.update(mat_n_layers=np.int32, mat_layer_d=np.float32, mat_layer_n=np.float32, mat_layer_k=np.float32)
        lm = int(np.asarray(sc["mat_layer_d"]).shape[1])
    for k, t in arrays.items():
        np.ascontiguousarray(sc[k], dtype=t).tofile(os.path.join(d, k + ".bin"))
    cam = sc["camera"]
    np.array(list(cam["eye"]) + list(cam["target"]) + [cam["fov_deg"], float(cam.get("ortho", False)),
                                                        cam.get("ortho_half_h", 1.0)], np.float64).tofile(
        os.path.join(d, "camera.bin"))
    meta = dict(n_verts=len(sc["verts"]), n_tris=len(sc["tris"]), n_lambda=len(sc["lambda_nm"]),
                n_mats=len(sc["mat_type"]), light_type=int(sc["light_type"]), light_mat=int(sc["light_mat"]),
                max_layers=lm)
    with open(os.path.join(d, "meta.txt"), "w") as f:
        for k, v in meta.items():
            f.write(f"{k} {v}\n")


def _check_run(cmd, env):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=600)
    report = r.stdout + r.stderr
    print(report[-2000:])
    assert r.returncode == 0, report[-4000:]
    for word in ("runtime error", "AddressSanitizer", "LeakSanitizer"):
        assert word not in report, report[-4000:]
    return r.stdout


@pytest.fixture(scope="module")
def scene_dirs(tmp_path_factory):
    base = tmp_path_factory.mktemp("scenes")
    out = {}
    for name, make in SCENES.items():
        _write_scene(make(), str(base / name))
        out[name] = str(base / name)
    return out


def test_oracle_under_sanitizers(scene_dirs, tmp_path):
    exe = str(tmp_path / "oracle_driver")
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                    os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(HERE, "oracle_driver.c"),
                    "-o", exe, "-lm"], check=True)
    for name, d in scene_dirs.items():
        out = _check_run([exe, d], SAN_ENV)
        assert "plain bvh=1" in out and "cache" in out and "window" in out and "probe finite" in out, name
        # the BVH and brute force give the same render
        lines = dict(l.split(" ", 1) for l in out.splitlines() if l.startswith("plain"))
        assert len({v.split(" rays")[0].split(" ", 1)[1] for v in lines.values()}) == 1, out


def _host_objects():
    need = [os.path.join(OBJ, f) for f in ("kernels.o", "bvh_device.o", "bvh_wide.o", "nrc.o")]
    if not all(os.path.exists(p) for p in need):
        from paper_1912_06474_amd import build
        build.build()
    return need


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="no hipcc")
def test_library_host_code_under_sanitizers(scene_dirs, tmp_path):
    hip_objs = _host_objects()
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-I", HERE]
    objs = []
    for src in (os.path.join(CSRC, "api.cpp"), os.path.join(CSRC, "bvh_build.cpp"),
                os.path.join(HERE, "host_driver.cpp")):
        o = str(tmp_path / (os.path.basename(src) + ".o"))
        subprocess.run(["hipcc", *flags, "-c", src, "-o", o], check=True, capture_output=True)
        objs.append(o)
    exe = str(tmp_path / "host_driver")
    clangxx = "/opt/rocm/llvm/bin/clang++"
    subprocess.run([clangxx, "-fsanitize=address,undefined", *objs, *hip_objs, "-L/opt/rocm/lib", "-lamdhip64",
                    "-Wl,-rpath,/opt/rocm/lib", "-o", exe], check=True)
    # the HIP runtime keeps allocations for the life of the process: leaks are not judged here
    env = dict(SAN_ENV, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0")
    for name, d in scene_dirs.items():
        out = _check_run([exe, d, str(tmp_path / f"tune_{name}.txt")], env)
        assert "host checks ok" in out, name
