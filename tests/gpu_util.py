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
    """Temporarily set environment variables read by the library at each call."""

    def __init__(self, **kv):
        self.kv = {k: str(v) for k, v in kv.items()}
        self.old = {}

    def __enter__(self):
        for k, v in self.kv.items():
            self.old[k] = os.environ.get(k)
            os.environ[k] = v

    def __exit__(self, *exc):
        for k, v in self.old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
