"""Build the CPU oracle library (test infrastructure only).

``python -m oracle.build`` or ``build()`` compiles ``oracle.c`` with gcc into
``oracle/liboracle.so``.  ``build(plant=N)`` compiles a copy with the N-th
planted mistake (see ``oracle.c``) into a separate file, used only by the
test that shows the pins catch a wrong oracle.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")


def lib_path(plant=None):
    if plant is None:
        return os.path.join(HERE, "liboracle.so")
    return os.path.join(HERE, f"liboracle_plant{int(plant)}.so")


def build(plant=None, out=None):
    out = out or lib_path(plant)
    cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", SRC,
           "-o", out + ".tmp"]
    if plant is not None:
        cmd.insert(1, f"-DORACLE_PLANT={int(plant)}")
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build())
