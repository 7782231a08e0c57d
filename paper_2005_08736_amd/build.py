"""Compile libhgks.so (HIP for gfx950) in-tree with hipcc."""
import concurrent.futures
import glob
import os
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhgks.so")
ARCH = os.environ.get("HGKS_OFFLOAD_ARCH", "gfx950")

# Packed FP32 arithmetic is switched off for every device function (the compiler
# would otherwise form v_pk_* FP32 instructions on its own).
HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def build(force: bool = True, verbose: bool = False, out: str = LIB, defines=()) -> str:
    deps = sources() + glob.glob(os.path.join(CSRC, "*.hpp")) + [os.path.join(HERE, "..", "include", "hgks.h")]
    if not force and os.path.exists(out) and os.path.getmtime(out) >= max(os.path.getmtime(d) for d in deps):
        return out
    # one object per source, compiled side by side, then one link
    flags = [f for f in HIPCC_FLAGS if f != "-shared"] + [f"-D{d}" for d in defines]
    with tempfile.TemporaryDirectory(prefix="hgks_build_") as tmpdir:
        objs, cmds = [], []
        for src in sources():
            obj = os.path.join(tmpdir, os.path.basename(src) + ".o")
            objs.append(obj)
            cmds.append(["hipcc", *flags, "-c", "-o", obj, src])
        workers = max(1, min(len(cmds), os.cpu_count() or 1, 8))
        with concurrent.futures.ThreadPoolExecutor(workers) as pool:
            for cmd, rc in zip(cmds, pool.map(_run, cmds)):
                if verbose:
                    print(" ".join(cmd))
                if rc != 0:
                    raise subprocess.CalledProcessError(rc, cmd)
        tmp = out + ".tmp"
        cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)
    return out


def _run(cmd) -> int:
    return subprocess.run(cmd).returncode


if __name__ == "__main__":
    print(build(verbose=True))
