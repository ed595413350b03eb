"""Host AddressSanitizer + UndefinedBehaviorSanitizer build of the ABI code.

The host parts of solver.cpp, fno.cpp and the line-FFT emulator are compiled with the
host sanitizers (-Xarch_host keeps the device code uninstrumented) and linked with the
kernel objects of the normal build into `tests/native/abi_host_checks.cpp`, which calls
every entry point that validates before touching a device (workspace sizes of every
supported grid, bad grids and parameters, batches, null handles, the surrogate's sizes)
and runs the FFT schedule against a direct DFT.  No device is used.
"""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
KERNEL_OBJS = [f"kern_{p}_{k}.o" for p in ("f64", "f32") for k in ("inv", "real", "fwd", "aux")] + [
    "finalize.o", "fno_fno_kernels.o"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, "\n".join([" ".join(cmd), r.stdout[-3000:], r.stderr[-3000:]])


def test_abi_and_fft_schedule_under_host_sanitizers(tmp_path):
    build = os.path.join(ROOT, "_build")
    if not all(os.path.exists(os.path.join(build, o)) for o in KERNEL_OBJS):
        from paper_2012_15133_amd import build as B
        B.build()
    if not os.path.exists(HIPCC) or shutil.which("g++") is None:
        pytest.skip("hipcc or g++ not available")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2012_15133_amd", "csrc"),
           "-I", os.path.join(ROOT, "paper_2012_15133_amd", "fno")]
    hip = [HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-fno-omit-frame-pointer", "-std=c++17", "-fPIC",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *inc,
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
    srcs = {"solver.o": "paper_2012_15133_amd/csrc/solver.cpp", "fno.o": "paper_2012_15133_amd/fno/fno.cpp",
            "emul.o": "tests/native/fft_emul.cpp"}
    procs = [subprocess.Popen(hip + ["-c", os.path.join(ROOT, s), "-o", str(tmp_path / o)],
                              stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True) for o, s in srcs.items()]
    for p in procs:
        out, _ = p.communicate(timeout=600)
        assert p.returncode == 0, out[-3000:]
    main = str(tmp_path / "main.o")
    _run(["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-I", os.path.join(ROOT, "include"),
          "-c", os.path.join(ROOT, "tests", "native", "abi_host_checks.cpp"), "-o", main])
    exe = str(tmp_path / "checks")
    _run(["g++", "-fsanitize=address,undefined", "-o", exe, main, *[str(tmp_path / o) for o in srcs],
          *[os.path.join(build, o) for o in KERNEL_OBJS], "-L/opt/rocm/lib", "-lamdhip64", "-lrocprofiler-sdk-roctx",
          "-Wl,-rpath,/opt/rocm/lib"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    print(r.stdout)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-5000:]
    assert "0 failures" in r.stdout
