"""Host-sanitized build of libstitch.so for the ABI tests: the same sources and device code,
with AddressSanitizer and UndefinedBehaviorSanitizer on the host code only (the argument
checking, planning and table building of stitch_api.cpp, pipe.cpp and the host halves of the
other files).  Run the tests against it with STITCH_LIB pointing at the result and the ASan
runtime preloaded (see asan_runtime())."""
from __future__ import annotations

import subprocess
from pathlib import Path

from .build import CSRC, HIPCC_FLAGS, ROOT, SOURCES, hipcc

OUT = Path(__file__).resolve().parent / "_build" / "libstitch_hostsan.so"
SAN = ["-O1", "-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-omit-frame-pointer"]


def asan_runtime() -> str:
    """Path of the ASan runtime shared library of the ROCm compiler (to LD_PRELOAD)."""
    clang = Path(hipcc()).resolve().parent.parent / "llvm" / "bin" / "clang"
    res = subprocess.run([str(clang), "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    return res.stdout.strip()


def build_sanitized() -> Path:
    OUT.parent.mkdir(parents=True, exist_ok=True)
    flags = [f for f in HIPCC_FLAGS if f != "-O3"] + SAN
    cmd = [hipcc(), *flags, f"-I{ROOT / 'include'}", f"-I{CSRC}", *map(str, SOURCES), "-o", str(OUT)]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("sanitized build failed:\n" + res.stdout + res.stderr)
    return OUT


if __name__ == "__main__":
    print(build_sanitized())
