"""Compiles the reference oracle (test infrastructure) with the host C compiler.

Three variants come out of the one source: the extended-precision oracle used by most checks; a
binary128 build for small lattices whose velocities are tiny enough that the extended build's
rounding approaches the fp64 parity bar; and an fp64 build that exists only to show the rounding
floor of the literal population form.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
BUILD_DIR = os.path.join(HERE, "_build")
SRC = os.path.join(HERE, "lbm_oracle.c")

VARIANTS = {
    "ld": ("liboracle.so", []),
    "fp64": ("liboracle_fp64.so", ["-DORACLE_FP64"]),
    "quad": ("liboracle_quad.so", ["-DORACLE_QUAD"]),
}


def lib_path(variant="ld"):
    return os.path.join(BUILD_DIR, VARIANTS[variant][0])


def build(force=True):
    """Compile both variants; with force=False only what is missing."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    for variant, (name, defs) in VARIANTS.items():
        out = os.path.join(BUILD_DIR, name)
        if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(SRC):
            continue
        tmp = out + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off", "-Wall",
               *defs, SRC, "-o", tmp, "-lm"] + (["-lquadmath"] if "-DORACLE_QUAD" in defs else [])
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)


if __name__ == "__main__":
    build()
    print("built", [lib_path(v) for v in VARIANTS])
