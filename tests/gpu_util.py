"""Helpers shared by the GPU tests (no method arithmetic here)."""
import os
import sys

import numpy as np

import oracle

ORACLE_OPS = [oracle.es_adjoint, oracle.es_apply, oracle.matern_cov_apply, oracle.matern_sample]
OP_NAMES = ["es_adjoint", "es_apply", "matern_cov_apply", "matern_sample"]
TOL = 1e-5  # relative L2 per result, FP32 GPU vs FP64 oracle


def rel_l2(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref)
    return np.linalg.norm(got - ref) / (den if den > 0 else 1.0)


def say(*a):
    """Name the case before a GPU step (so a fault leaves a trace)."""
    print(*a, file=sys.stderr, flush=True)


class env:
    """Temporarily set environment variables read by the library at each call.

    Only names the test session created before the first device call (conftest.KNOBS) may be
    set here, and they are restored to a value, never removed: adding or removing a name can
    reallocate the process's environment array while a runtime thread reads it (getenv), so
    that is done only before any thread of the device runtime exists.  The library reads an
    empty knob as an absent one.
    """

    def __init__(self, **kv):
        self.kv = {k: str(v) for k, v in kv.items()}
        self.old = {}

    def __enter__(self):
        for k, v in self.kv.items():
            if k not in os.environ:
                raise KeyError(f"{k} was not created before the first device call (add it to conftest.KNOBS)")
            self.old[k] = os.environ[k]
            os.environ[k] = v

    def __exit__(self, *exc):
        for k, v in self.old.items():
            os.environ[k] = v
