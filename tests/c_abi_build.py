"""Build tests/_bin/c_abi_program, a plain C client of the library used by the
C-ABI test (gcc; links libnematic_sph.so from the package directory)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
OUT = os.path.join(HERE, "_bin", "c_abi_program")


def build() -> str:
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    cmd = ["gcc", "-O2", "-Wall", "-Wextra", "-std=c11", os.path.join(HERE, "c_abi_program.c"),
           "-I", os.path.join(ROOT, "include"), "-L", os.path.join(ROOT, "paper_2108_08919_amd"),
           "-lnematic_sph", "-Wl,-rpath,$ORIGIN/../../paper_2108_08919_amd", "-o", OUT]
    subprocess.run(cmd, check=True)
    return OUT


if __name__ == "__main__":
    print(build())
