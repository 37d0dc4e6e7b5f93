"""Builds of the oracle and of the library's host code with AddressSanitizer and
UndefinedBehaviorSanitizer (CPU test infrastructure; the device code is built as usual).

oracle_sanitized():  oracle/mlmc_oracle.c + oracle_sanitize.c, gcc, OpenMP.
plan_sanitized():    the library's plan construction (csrc/abi.hip with the kernels it
                     launches, and csrc/proposal.hip, whose training the learned run calls)
                     + plan_sanitize.cpp, hipcc with the sanitizers on the host pass.
"""
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(ROOT, "_build")
HOST_SAN = "-fsanitize=address,undefined"


def oracle_sanitized() -> str:
    os.makedirs(OUT, exist_ok=True)
    exe = os.path.join(OUT, "oracle_sanitize")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-ffp-contract=off", HOST_SAN,
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-o", exe + ".tmp",
           os.path.join(ROOT, "oracle", "mlmc_oracle.c"), os.path.join(HERE, "oracle_sanitize.c"),
           "-lm"]
    subprocess.check_call(cmd)
    os.replace(exe + ".tmp", exe)
    return exe


def plan_sanitized() -> str | None:
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        return None
    os.makedirs(OUT, exist_ok=True)
    exe = os.path.join(OUT, "plan_sanitize")
    csrc = os.path.join(ROOT, "paper_1904_12754_amd", "csrc")
    host = ["-Xarch_host", HOST_SAN, "-Xarch_host", "-fno-sanitize-recover=all"]
    cmd = [hipcc, "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "--offload-arch=gfx950",
           *host, "-I", os.path.join(ROOT, "include"), "-o", exe + ".tmp",
           os.path.join(csrc, "abi.hip"), os.path.join(csrc, "kernels.hip"),
           os.path.join(csrc, "proposal.hip"), os.path.join(HERE, "plan_sanitize.cpp")]
    subprocess.check_call(cmd, stderr=subprocess.DEVNULL)
    os.replace(exe + ".tmp", exe)
    return exe
