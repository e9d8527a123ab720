"""FP64 reference oracle for the ray-Born single-step inversion.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from here.  The GPU
library shares no code with this package: the two are separate
implementations of the same definitions, checked against each other.

Layout:

* ``raytrace.c`` / ``rays.py`` - RK4 ray fans through a bilinear slowness
  grid, ray-tube spreading, first-arrival ray-to-grid interpolation (paper,
  Forward Problem section, Eqs. 4-7), in plain C (gcc, FP64, no FMA);
* ``born.py`` - Green's functions on the tables (Eqs. 4-5) and the Born
  forward operator, its adjoint and the diagonal of the Gauss-Newton
  Hessian (Inverse Problem section, Eqs. 8-10), in NumPy FP64;
* ``invert.py`` - data-space weights (receiver selection and outlier
  zeroing, Results section), the diagonally weighted single step, the
  Jacobi-preconditioned CG solution of the linear subproblem and the
  low-to-high frequency sweep (Inverse Problem section).

Where the paper leaves a choice open, the reading taken is stated in the
docstring of the function that implements it.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "_liboracle.so")
SRC = os.path.join(HERE, "raytrace.c")


def build(force: bool = True) -> str:
    """Compile the C part of the oracle with gcc (FP64, no FMA contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-fPIC", "-shared", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB
