"""Build the CPU oracle libraries with gcc.

TEST INFRASTRUCTURE ONLY.  Produces, next to this file:
  liboracle_f64.so   oracle arithmetic in double
  liboracle_ld.so    oracle arithmetic in long double (x87 80-bit)
Both are compiled without fast-math and with -ffp-contract=off so that every
product and sum is rounded exactly as written.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
VARIANTS = {
    "f64": ("double", "liboracle_f64.so"),
    "ld": ("long double", "liboracle_ld.so"),
}


def lib_path(variant):
    return os.path.join(HERE, VARIANTS[variant][1])


def build(force=True, verbose=False):
    """Compile both variants; with force=False only missing libraries are built."""
    for variant, (real, name) in VARIANTS.items():
        out = os.path.join(HERE, name)
        if not force and os.path.exists(out):
            continue
        cmd = [
            "gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
            "-fno-fast-math", "-Wall", "-Wextra", f"-DORACLE_REAL={real}",
            SRC, "-o", out + ".tmp", "-lm",
        ]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True, cwd=HERE)
        os.replace(out + ".tmp", out)


if __name__ == "__main__":
    build(force=True, verbose=True)
