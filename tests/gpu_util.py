"""Shared helpers for the GPU parity tests (device setup and error metrics)."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def device_or_skip():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_04755_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2009_04755_amd import build
        build.build()
    return torch.device("cuda", 0)


def announce(msg: str):
    sys.stdout.write("[gpu-case] %s\n" % msg)
    sys.stdout.flush()


def floored_rel(got, ref, floor):
    """|got - ref| / max(|ref|, floor): the pass metric for signed sums near zero."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return np.abs(got - ref) / np.maximum(np.abs(ref), floor)


def upper_to_dense(packed, n):
    iu = np.triu_indices(n, 1)
    out = np.zeros((n, n))
    out[iu] = packed
    return out
