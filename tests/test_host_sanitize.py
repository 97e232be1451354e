"""The host side of the library (C ABI, index file, CL map, trainers, tuning
table) built with AddressSanitizer and UndefinedBehaviorSanitizer and driven
by tests/host_checks.cpp, including forced host allocation failures.  CPU
only: no call reaches the GPU.  The device code is linked from the regular
build, unsanitised."""
import glob
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2606_07156_amd", "csrc")
BUILD = os.path.join(ROOT, "paper_2606_07156_amd", "_build")
HOST_SRC = ("capi.cpp", "train.cpp", "build.cpp", "clmap.cpp", "server.cpp", "tune.cpp")
DEVICE_OBJ = ("kernels.hip.o", "scan_ph1.hip.o", "scan_ph2.hip.o", "scan_ph3.hip.o", "cl.hip.o", "noalloc.hip.o")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def _hip_lib_dir():
    try:
        import importlib.util
        spec = importlib.util.find_spec("torch")
        d = os.path.join(list(spec.submodule_search_locations)[0], "lib")
        if glob.glob(os.path.join(d, "libamdhip64.so*")):
            return d
    except Exception:
        pass
    return os.path.join(ROCM, "lib")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no g++")
def test_host_side_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    objs = [os.path.join(BUILD, o) for o in DEVICE_OBJ]
    if not all(os.path.exists(o) for o in objs):
        pytest.skip("device objects not built (run paper_2606_07156_amd/build.py)")
    san = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined"]
    flags = ["-std=c++17", "-O1", "-g", "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROCM, "include")] + san
    host_objs = []
    for src in HOST_SRC:
        o = str(tmp_path / (src + ".o"))
        r = subprocess.run(["g++", *flags, "-c", "-o", o, os.path.join(CSRC, src)], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
        host_objs.append(o)
    exe = str(tmp_path / "host_checks")
    libdir = _hip_lib_dir()
    r = subprocess.run(["g++", *flags, "-o", exe, os.path.join(HERE, "host_checks.cpp"), *host_objs, *objs,
                        "-L" + libdir, "-l:libamdhip64.so", "-Wl,-rpath," + libdir, "-pthread"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:allocator_may_return_null=1:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([exe, str(tmp_path)], capture_output=True, text=True, env=env, timeout=600)
    out = r.stdout + r.stderr
    if r.returncode != 0 and "LeakSanitizer does not work under ptrace" in out:
        env["ASAN_OPTIONS"] = env["ASAN_OPTIONS"].replace("detect_leaks=1", "detect_leaks=0")
        r = subprocess.run([exe, str(tmp_path)], capture_output=True, text=True, env=env, timeout=600)
        out = r.stdout + r.stderr
    assert r.returncode == 0, out[-6000:]
    assert "host checks: ok" in out
