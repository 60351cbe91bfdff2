"""Helpers for the GPU parity tests (the oracle is the reference)."""
import numpy as np
import pytest
import torch

TOL = {0: 1e-12, 1: 1e-5, 2: 4e-3, 3: 3e-2}  # relative-norm bounds per storage precision (F64, F32, F16, BF16)
PREC_NAME = {0: "f64", 1: "f32", 2: "f16", 3: "bf16"}


def gpu_available():
    return torch.cuda.is_available()


def np_of(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def on_parity(field, mask):
    extra = field.ndim - 4
    return np.where(mask.reshape(mask.shape + (1,) * extra), field, 0)


@pytest.fixture(scope="module")
def ctx():
    if not gpu_available():
        pytest.skip("no GPU")
    from paper_1109_2935_amd import lqcd as L
    c = L.lqcd_context_create()
    yield c
    torch.cuda.synchronize()
    L.lqcd_context_destroy(c)
