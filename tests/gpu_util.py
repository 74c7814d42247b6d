"""Helpers for the GPU tests: device transfer and error metrics."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no ROCm GPU")


def to_dev(a, dtype=torch.float64):
    t = torch.from_numpy(np.asfortranarray(a)).to(dtype)
    return t.to("cuda:0")


def to_np(t):
    return np.asfortranarray(t.detach().cpu().to(torch.float64).numpy())


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def announce(name, **kw):
    print("CASE %s %s" % (name, " ".join("%s=%s" % kv for kv in kw.items())), flush=True)
