"""Build the oracle shared library (test infrastructure only).

The oracle is plain C++17 compiled with the host compiler; it never touches the
GPU and shares no source with the HIP library.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hgks_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")


LIB_SANITIZED = os.path.join(HERE, "liboracle_asan.so")
# AddressSanitizer and UndefinedBehaviorSanitizer build: every report aborts
SANITIZE_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]


def build(force: bool = True, sanitize: bool = False) -> str:
    """Compile oracle/liboracle.so (or, with sanitize, the ASan + UBSan build
    oracle/liboracle_asan.so, which must be loaded into a process that preloads
    the sanitizer runtimes); returns its path."""
    out = LIB_SANITIZED if sanitize else LIB
    deps = [SRC] + [os.path.join(HERE, h) for h in ("dual.hpp", "counting.hpp")]
    if not force and os.path.exists(out) and os.path.getmtime(out) >= max(os.path.getmtime(d) for d in deps):
        return out
    tmp = out + ".tmp"
    opt = ["-O1"] + SANITIZE_FLAGS if sanitize else ["-O2"]
    cmd = ["g++", *opt, "-std=c++17", "-fopenmp", "-shared", "-fPIC", "-o", tmp, SRC]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def sanitizer_runtimes() -> list:
    """Paths of the ASan and UBSan runtimes of the host compiler (for LD_PRELOAD)."""
    libs = []
    for name in ("libasan.so", "libubsan.so"):
        path = subprocess.run(["g++", f"-print-file-name={name}"], check=True, capture_output=True,
                              text=True).stdout.strip()
        libs.append(path)
    return libs


if __name__ == "__main__":
    print(build())
