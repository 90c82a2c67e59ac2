"""Builds the host-only serving test harness with g++ (no HIP): the scheduler
of paper_2405_07122_amd/csrc/pcf_serve_core.cpp with a host-memory executor,
as a shared library for ctypes and as a thread-sanitized stress program."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2405_07122_amd", "csrc")
OUT = os.path.join(HERE, "_build")
CORE = os.path.join(CSRC, "pcf_serve_core.cpp")
MOCK = os.path.join(HERE, "mock_executor.cpp")


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(" ".join(cmd) + "\n" + r.stdout + r.stderr)


def build_lib() -> str:
    os.makedirs(OUT, exist_ok=True)
    lib = os.path.join(OUT, "libpcfserve_mock.so")
    _run(["g++", "-O1", "-g", "-std=c++17", "-fPIC", "-shared", "-I", CSRC, CORE, MOCK, "-o", lib,
          "-lpthread"])
    return lib


def build_stress(sanitize: str | None = "thread") -> str:
    os.makedirs(OUT, exist_ok=True)
    exe = os.path.join(OUT, f"stress_{sanitize or 'plain'}")
    flags = [f"-fsanitize={sanitize}"] if sanitize else []
    _run(["g++", "-O1", "-g", "-std=c++17", *flags, "-I", CSRC, CORE, MOCK,
          os.path.join(HERE, "stress.cpp"), "-o", exe, "-lpthread"])
    return exe


if __name__ == "__main__":
    print(build_lib())
    print(build_stress())
