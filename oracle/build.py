"""Builds the CPU oracle (test infrastructure) into oracle/liboracle.so with gcc."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
CMD = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared", "-pthread",
       os.path.join(HERE, "oracle.c"), "-o", LIB]


def build() -> str:
    subprocess.run(CMD, check=True)
    return LIB


if __name__ == "__main__":
    print(build())
