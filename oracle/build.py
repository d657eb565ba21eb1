"""Compile the CPU oracle (plain C, FP64, OpenMP) into oracle/liboracle.so.

Test infrastructure: building the checker is not using it.
"""
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))


def build(verbose: bool = False) -> str:
    out = os.path.join(_HERE, "liboracle.so")
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
           os.path.join(_HERE, "hisq_oracle.c"), "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build_timing(out_dir: str, verbose: bool = False) -> str:
    """The oracle built -O3 for the machine it runs on (-march=native), into `out_dir`: the build the
    benchmark's CPU baseline times.  Falls back to -O3 without -march if the compiler refuses.  The same
    source as the checker; only the code generation differs."""
    os.makedirs(out_dir, exist_ok=True)
    out = os.path.join(out_dir, "liboracle_timing.so")
    for arch in (["-march=native"], []):
        cmd = ["gcc", "-O3"] + arch + ["-fopenmp", "-fPIC", "-shared", "-std=c99",
                                       os.path.join(_HERE, "hisq_oracle.c"), "-o", out, "-lm"]
        if verbose:
            print(" ".join(cmd))
        if subprocess.run(cmd, capture_output=True).returncode == 0:
            return out
    raise RuntimeError("cannot build the oracle timing library")


if __name__ == "__main__":
    print(build(verbose=True))
