"""Build bn_c_check (the C ABI driven from plain C) against the in-tree libbn.so with gcc."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
BIN = os.path.join(HERE, "bn_c_check")


def build(verbose: bool = True) -> str:
    cmd = [os.environ.get("CC", "gcc"), "-O2", "-std=c11", "-Wall", "-Wextra", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"),
           os.path.join(HERE, "bn_c_check.c"),
           "-L", os.path.join(ROOT, "paper_2604_21566_amd"), "-lbn", "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
           "-Wl,-rpath,$ORIGIN/../../paper_2604_21566_amd", "-Wl,-rpath," + os.path.join(ROCM, "lib"),
           "-o", BIN + ".tmp"]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError(f"gcc failed for bn_c_check.c:\n{p.stdout}\n{p.stderr}")
    os.replace(BIN + ".tmp", BIN)
    if verbose:
        print(f"built {BIN}")
    return BIN


if __name__ == "__main__":
    build()
