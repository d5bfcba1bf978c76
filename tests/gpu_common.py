"""Shared helpers of the GPU parity tests."""

import sys

import numpy as np
import pytest
import torch


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def lib():
    need_gpu()
    import paper_2210_16435_amd as sf

    return sf


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_np(t):
    return t.detach().cpu().numpy()


def eig_parity(lam_gpu, lam_ref, rtol):
    """Relative eigenvalue error, the trivial pair against lambda_2."""
    lam_gpu = np.asarray(lam_gpu)
    lam_ref = np.asarray(lam_ref)
    err = np.abs(lam_gpu - lam_ref)
    scale = np.maximum(np.abs(lam_ref), np.abs(lam_ref[1]) if lam_ref.size > 1 else 1.0)
    return float((err / scale).max())
