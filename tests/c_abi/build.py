"""Build the plain-C client of liblbm (c_abi_check.c) next to its source, with
gcc in C11 mode against the HIP runtime's C interface.  Called by the
repository's build step after the library; the binary finds liblbm.so through
an rpath relative to itself."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
SRC = os.path.join(HERE, "c_abi_check.c")
OUT = os.path.join(HERE, "c_abi_check")


def build() -> str:
    lib_dir = os.path.join(ROOT, "paper_2101_11856_amd")
    rel = os.path.relpath(lib_dir, HERE)
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-Wextra", "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include",
           f"-I{os.path.join(ROOT, 'include')}", SRC, "-o", OUT, f"-L{lib_dir}", "-llbm", f"-L{ROCM}/lib",
           "-lamdhip64", "-lm", f"-Wl,-rpath,$ORIGIN/{rel}", f"-Wl,-rpath,{ROCM}/lib"]
    subprocess.check_call(cmd)
    return OUT


if __name__ == "__main__":
    print("built", build())
