"""Build the CPU oracle (test infrastructure) into oracle/liboracle.so with gcc.

``build(sanitize=True)`` builds oracle/liboracle_san.so instead, with
AddressSanitizer and UndefinedBehaviorSanitizer (errors abort), for a CPU run
of the oracle's pins under the sanitizers; ``oracle`` loads it when the
environment variable MPC_ORACLE_LIB names it."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
OUT = os.path.join(HERE, "liboracle.so")
OUT_SAN = os.path.join(HERE, "liboracle_san.so")
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]


def build(verbose: bool = False, sanitize: bool = False) -> str:
    out = OUT_SAN if sanitize else OUT
    cmd = ["gcc", "-O1" if sanitize else "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
           *(SAN_FLAGS if sanitize else []), SRC, "-o", out + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv))
