"""Host sanitizer runs: the C oracle built with AddressSanitizer and
UndefinedBehaviorSanitizer (gcc, every check fatal, leak detection on) and
driven through every exported routine on small and degenerate inputs
(tests/sanitize_oracle.c)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "sanitize_oracle")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(HERE, "sanitize_oracle.c"), os.path.join(ROOT, "oracle", "oracle.c"),
           "-o", exe, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=99",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "sanitize_oracle: ok" in r.stdout


def _abi_sanitize_exe():
    """The library's sources and tests/sanitize_abi.cpp compiled with the
    host side instrumented (device code is unaffected), linked into one
    executable; cached under _build/sanitize by a digest of the sources."""
    import concurrent.futures as cf
    import glob
    import hashlib
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    clang = "/opt/rocm/llvm/bin/clang++"
    if not (os.path.exists(hipcc) and os.path.exists(clang)):
        pytest.skip("ROCm compilers not found")
    srcs = sorted(glob.glob(os.path.join(ROOT, "paper_2310_03341_amd", "csrc", "*.hip")))
    drv = os.path.join(HERE, "sanitize_abi.cpp")
    deps = srcs + glob.glob(os.path.join(ROOT, "paper_2310_03341_amd", "csrc", "*.h")) + \
        [drv, os.path.join(ROOT, "include", "bdg.h")]
    h = hashlib.sha256()
    for f in sorted(deps):
        h.update(open(f, "rb").read())
    out = os.path.join(ROOT, "_build", "sanitize", h.hexdigest()[:16])
    exe = os.path.join(out, "sanitize_abi")
    if os.path.exists(exe):
        return exe
    os.makedirs(out, exist_ok=True)
    flags = ["--offload-arch=gfx950", "-O3", "-g", "-fPIC", "-std=c++17",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I" + os.path.join(ROOT, "include"),
             "-Xarch_host", "-fsanitize=address,undefined",
             "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]

    def comp(src):
        obj = os.path.join(out, os.path.basename(src) + ".o")
        r = subprocess.run([hipcc] + flags + ["-c", src, "-o", obj], capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(r.stderr[-4000:])
        return obj
    with cf.ThreadPoolExecutor(8) as ex:
        objs = list(ex.map(comp, srcs + [drv]))
    tmp = exe + ".tmp"
    r = subprocess.run([clang, "-fsanitize=address,undefined", "-o", tmp] + objs +
                       ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(r.stderr[-4000:])
    os.replace(tmp, exe)
    return exe


def test_abi_host_code_under_asan_and_ubsan():
    exe = _abi_sanitize_exe()
    # leak checking is off: the HIP runtime keeps allocations until exit
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:exitcode=99",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert "sanitize_abi: ok" in r.stdout
