"""Build the plain C client of the decoder's C ABI (tests/c_client/decode_client)
with gcc: it links libqkdldpc.so and the HIP runtime and uses nothing else."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
BINARY = os.path.join(HERE, "decode_client")


def build(verbose: bool = False) -> str:
    pkg = os.path.join(ROOT, "paper_1903_10107_amd")
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-D__HIP_PLATFORM_AMD__",
           f"-I{ROCM}/include", f"-I{os.path.join(ROOT, 'include')}",
           os.path.join(HERE, "decode_client.c"), "-o", BINARY + ".tmp",
           f"-L{pkg}", "-lqkdldpc", f"-L{ROCM}/lib", "-lamdhip64",
           # the library is found next to the checkout wherever it is copied
           "-Wl,-rpath,$ORIGIN/../../paper_1903_10107_amd", f"-Wl,-rpath,{ROCM}/lib"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("C client build failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    os.replace(BINARY + ".tmp", BINARY)
    return BINARY


if __name__ == "__main__":
    print(build(verbose=True))
