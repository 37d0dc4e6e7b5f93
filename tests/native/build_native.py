"""Build the host-side helper programs the CPU tests use (not GPU code).

rocrand_philox_ref: rocRAND's Philox4x32-10 engine run on the host, an implementation
independent of the oracle's, used to pin the oracle's generator.
"""
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(ROOT, "_build")


def rocrand_ref(force: bool = False) -> str | None:
    src = os.path.join(HERE, "rocrand_philox_ref.cpp")
    exe = os.path.join(OUT, "rocrand_philox_ref")
    if not force and os.path.exists(exe) and os.path.getmtime(exe) >= os.path.getmtime(src):
        return exe
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        return None
    os.makedirs(OUT, exist_ok=True)
    subprocess.check_call([hipcc, "-O1", "-o", exe + ".tmp", src])
    os.replace(exe + ".tmp", exe)
    return exe


def log_bound(force: bool = False) -> str | None:
    """GPU program checking the fast holding-time log bracket over all 2^32 words."""
    src = os.path.join(HERE, "log_bound.hip")
    dep = os.path.join(ROOT, "paper_1904_12754_amd", "csrc", "common.h")
    exe = os.path.join(OUT, "log_bound")
    if (not force and os.path.exists(exe)
            and os.path.getmtime(exe) >= max(os.path.getmtime(src), os.path.getmtime(dep))):
        return exe
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        return None
    os.makedirs(OUT, exist_ok=True)
    subprocess.check_call([hipcc, "-O3", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                           "--offload-arch=gfx950", "-o", exe + ".tmp", src],
                          stderr=subprocess.DEVNULL)
    os.replace(exe + ".tmp", exe)
    return exe


if __name__ == "__main__":
    print(rocrand_ref(force=True))
    print(log_bound(force=True))


def driver_hook(force: bool = False) -> str | None:
    """Host program checking Algorithm 1's driver and its after-pilot hook on a mock."""
    src = os.path.join(HERE, "driver_hook.cpp")
    deps = [src, os.path.join(ROOT, "paper_1904_12754_amd", "csrc", "driver.h"),
            os.path.join(ROOT, "include", "mlmc_expv.h")]
    exe = os.path.join(OUT, "driver_hook")
    if (not force and os.path.exists(exe)
            and os.path.getmtime(exe) >= max(os.path.getmtime(d) for d in deps)):
        return exe
    gxx = shutil.which("g++")
    if gxx is None:
        return None
    os.makedirs(OUT, exist_ok=True)
    subprocess.check_call([gxx, "-O1", "-std=c++17", "-Wall", "-o", exe + ".tmp", src])
    os.replace(exe + ".tmp", exe)
    return exe
