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


# A single wrong site is diluted in a whole-field norm (one site of 2048 is 2%
# of it), so every operator check also bounds the worst site: its error norm
# relative to the RMS site norm of the reference (sites where the reference is
# non-zero). For independent rounding errors the largest of a few thousand
# site errors is about 3x their RMS; SITE_FACTOR leaves room for that.
SITE_FACTOR = 4.0
MEASURED = []  # (test id, kind, value, bound), written to gpurun_out/ by conftest


def site_err(a, b):
    inner = 12 if b.shape[-2:] == (4, 3) else b.shape[-1]
    d = np.linalg.norm((a - b).reshape(-1, inner), axis=1)
    nb = np.linalg.norm(b.reshape(-1, inner), axis=1)
    nz = nb > 0
    rms = np.sqrt(np.mean(nb[nz] ** 2)) if nz.any() else 1.0
    return float(d.max() / rms)


def check(got, ref, bound, what=""):
    """Assert the whole-field relative error and the worst-site error (see
    SITE_FACTOR) against `bound`; record both."""
    import os
    e, es = rel(got, ref), site_err(got, ref)
    test = os.environ.get("PYTEST_CURRENT_TEST", "?").split(" ")[0]
    MEASURED.append((test + (" " + what if what else ""), float(e), es, bound))
    assert e < bound, (what, "norm", e, bound)
    assert es < SITE_FACTOR * bound, (what, "site", es, SITE_FACTOR * bound)
    return e


def check_entries(got, ref, bound, what=""):
    """As check, for a weight gradient: whole-tensor relative error, and the
    worst single complex entry relative to the RMS entry of the reference."""
    import os
    e = rel(got, ref)
    rms = np.sqrt(np.mean(np.abs(ref) ** 2))
    es = float(np.abs(got - ref).max() / (rms if rms > 0 else 1.0))
    test = os.environ.get("PYTEST_CURRENT_TEST", "?").split(" ")[0]
    MEASURED.append((test + (" " + what if what else ""), float(e), es, bound))
    assert e < bound, (what, "norm", e, bound)
    assert es < SITE_FACTOR * bound, (what, "entry", es, SITE_FACTOR * bound)
    return e


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
