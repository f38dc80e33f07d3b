"""A second valid FP64 evaluation of the oracle, for tests only.

The oracle (``oracle/hps.py``) solves every leaf and merge system with LU factors kept
from the build.  The GPU library instead forms explicit inverses (A_ii^{-1}, X) so that
its solve is pure matrix-vector streaming.  Both are exact in exact arithmetic; in FP64
they round differently, and the difference between them measures how far apart two
correct FP64 evaluations of the same discrete solution can be at a given size (the
conditioning floor of I - gamma dt L_h).

``explicit_inverses()`` is a context manager that makes the oracle use explicit
inverses (LAPACK getrf + getri through ``numpy.linalg.inv``) in place of its LU solves,
without changing any other step.  It lives here, not in ``oracle/``, because it is a
measuring device for tolerances, not part of the oracle.
"""
import contextlib
import types

import numpy as np


def _inv(a):
    return np.linalg.inv(a)


def _apply(inv, b):
    return inv @ b


@contextlib.contextmanager
def explicit_inverses():
    import oracle.hps as oh
    saved = oh.sla
    oh.sla = types.SimpleNamespace(lu_factor=_inv, lu_solve=_apply)
    try:
        yield
    finally:
        oh.sla = saved
