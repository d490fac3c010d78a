"""Compile the generator library (host C++, OpenMP) in place."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "graphgen.cpp")
LIB = os.path.join(HERE, "libgraphgen.so")


def build(verbose: bool = False) -> str:
    cmd = ["g++", "-O3", "-std=c++17", "-fopenmp", "-fPIC", "-shared", SRC, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB
