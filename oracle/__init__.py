"""Oracle for the segmented block Cholesky KKT solver -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct CPU implementation of what the GPU path computes,
written from the paper (arXiv 2511.00946, "Parallel KKT Solver in PIQP for
Multistage Optimization") and shared with nothing in the product package.  Only
``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it; the product library never does.

Modules
  ``blockchol``  ctypes wrapper of ``block_chol.c``: right-looking block Cholesky
                 and triangular solves on a grid of dense blocks (any block order).
  ``kkt``        the block-tridiagonal-arrow KKT matrix of Eq. (3), its permuted
                 order (Sec. 3.1), factor / solve / adjoint / residual.
  ``partition``  the segment-length rule of Eq. (13) and the complexity model
                 (O_par, O_seq, speedup gamma) behind Table 2.
  ``flops``      per-phase flop counts of Algorithms 1-3 under the paper's
                 counting convention (Table 1).
"""
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "block_chol.c")
_LIB = os.path.join(_HERE, "_build", "libblockchol.so")


def build(force=False):
    """Compile ``block_chol.c`` with gcc (-O2, IEEE arithmetic, no fast-math)."""
    if (not force and os.path.exists(_LIB)
            and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC)):
        return _LIB
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off",
                           "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def library_path():
    return build(force=False)
