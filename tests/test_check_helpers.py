"""CPU pins of the GPU tests' own check helpers: the torch evaluation of the
oracle's Psi (used where the numpy oracle is too slow for full-size checks)
must equal the oracle's RHSketch, and the condition-number and orthogonality
helpers must equal their numpy definitions."""
import numpy as np
import pytest

from oracle import sketch as osk, metrics
from tests.gpu_util import psi_apply_torch, cond_gram, orth_err


@pytest.mark.parametrize("kind", ["srht", "gauss"])
@pytest.mark.parametrize("n,m,l", [(5000, 7, 96), (4096, 12, 4096 - 12), (3, 1, 2)])
def test_psi_apply_torch_equals_oracle(kind, n, m, l):
    torch = pytest.importorskip("torch")
    if kind == "gauss" and l > 512:
        l = 512
    sk = osk.Sketch(osk.SRHT if kind == "srht" else osk.GAUSS, n, m, l, seed=5)
    X = np.random.default_rng(1).standard_normal((n, 37))
    ref = osk.rh_sketch(X, sk)
    got = psi_apply_torch(sk, torch.from_numpy(X), chunk=16).numpy()
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_psi_apply_torch_exact_on_integers():
    """Integer inputs: every butterfly sum is an exact integer, so the torch
    evaluation equals the oracle bit for bit up to the two power-of-two-free
    scalings (compared before scaling by multiplying back)."""
    torch = pytest.importorskip("torch")
    n, m, l = 1 << 12, 4, 64
    sk = osk.Sketch(osk.SRHT, n, m, l, seed=2)
    X = np.random.default_rng(3).integers(-3, 4, size=(n, 5)).astype(np.float64)
    ref = osk.rh_sketch(X, sk)
    got = psi_apply_torch(sk, torch.from_numpy(X)).numpy()
    assert np.array_equal(got[:m], ref[:m])
    assert np.max(np.abs(got - ref)) <= 1e-14 * np.max(np.abs(ref))


def test_cond_and_orth_helpers():
    torch = pytest.importorskip("torch")
    A = np.random.default_rng(4).standard_normal((300, 9)) @ np.diag(np.logspace(0, -3, 9))
    assert abs(cond_gram(torch.from_numpy(A)) - metrics.cond(A)) <= 1e-9 * metrics.cond(A)
    Q, _ = np.linalg.qr(A)
    assert orth_err(torch.from_numpy(Q)) == pytest.approx(metrics.orth_error(Q), abs=1e-15)
