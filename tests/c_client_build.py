"""Compiles tests/c_client.c (a plain C99 client of include/mfh.h) with gcc
against the built library; used by the CPU and GPU tests of the client."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build_client(out_dir):
    """Returns the path of the compiled client (raises on a compiler error)."""
    libdir = os.path.join(ROOT, "paper_1904_13131_amd")
    exe = os.path.join(out_dir, "c_client")
    cmd = ["gcc", "-std=c99", "-O1", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"),
           os.path.join(ROOT, "tests", "c_client.c"), "-L", libdir, "-lmfh",
           "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
           f"-Wl,-rpath,{libdir}", f"-Wl,-rpath,{os.path.join(ROCM, 'lib')}", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode:
        raise RuntimeError(f"c_client build failed:\n{r.stderr[-3000:]}")
    return exe
