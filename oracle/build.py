"""Builds oracle/liboracle.so with gcc (plain C, OpenMP, no fast-math)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def build(force: bool = True) -> str:
    src = os.path.join(HERE, "sv_oracle.c")
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(src):
        tmp = LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
                        "-std=c99", "-Wall", "-o", tmp, src], check=True)
        os.replace(tmp, LIB)
    return LIB


def build_sanitized(driver_src, out_dir):
    """The oracle and a driver `driver_src` compiled together with
    AddressSanitizer and UndefinedBehaviorSanitizer; returns the binary."""
    os.makedirs(out_dir, exist_ok=True)
    exe = os.path.join(out_dir, "oracle_driver")
    subprocess.run(["gcc", "-O1", "-g", "-fno-fast-math", "-fopenmp", "-std=c99", "-Wall",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
                    "-o", exe, os.path.join(HERE, "sv_oracle.c"), driver_src, "-lm"], check=True)
    return exe


if __name__ == "__main__":
    print(build())
