"""The threshold certificate's mathematics, on the CPU.

The kept-column t-SVT certifies that the columns R left below tau have
spectral norm <= tau through, with H = R^T R / tau^2,
    (sigma_max(R) / tau)^16 = lambda_max(H)^8 <= trace(H^8) = ||H^4||_F^2,
computed in FP32 from the Gram matrix with two squarings, and passes a slice
iff ||H^4||_F^2 <= (1 - delta)^8 with
    delta = 2 (m + 2 p) 2^-24 trace(H) + 2^-8.
Checked here in numpy, with FP32 rounding where the GPU rounds:
  * the inequality on spectra from one dominant value to many equal ones;
  * soundness of the rule: it never passes when sigma_max(R) > tau, including
    just above tau and with many singular values near the largest;
  * usefulness: it passes with a gap (sigma_max(R) <= 0.8 tau, few values
    near the largest), and fails at the continuum edge, as the mode expects.
"""
import numpy as np
import pytest


def certificate_passes(R, tau):
    """The rule, with the GPU's precisions: R / tau rounded to FP32, Gram
    matrix and squarings in FP32, sum of squares and margin in FP64."""
    m, p = R.shape
    As = (R / tau).astype(np.float32)
    H = As.T @ As
    H2 = H @ H
    H4 = H2 @ H2
    S = float(np.sum(H4.astype(np.float64) ** 2))
    tr = float(np.sum(R.astype(np.float64) ** 2)) / tau**2
    delta = 2.0 * (m + 2.0 * p) * 2.0**-24 * tr + 2.0**-8
    return delta < 1.0 and S <= (1.0 - delta) ** 8


def with_spectrum(rng, m, p, s):
    """An m x p matrix with singular values s (descending, len <= p)."""
    U, _ = np.linalg.qr(rng.standard_normal((m, len(s))))
    V, _ = np.linalg.qr(rng.standard_normal((p, len(s))))
    return (U * s) @ V.T


@pytest.mark.parametrize("kind", ["one", "few", "flat", "marchenko"])
def test_schatten_inequality(kind):
    rng = np.random.default_rng(11)
    n = 64
    if kind == "one":
        lam = np.r_[1.0, 1e-3 * rng.random(n - 1)]
    elif kind == "few":
        lam = np.r_[np.ones(4), 0.5 * rng.random(n - 4)]
    elif kind == "flat":
        lam = np.ones(n)
    else:
        lam = np.sort(rng.random(n) ** 2)[::-1]
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    H = (Q * lam) @ Q.T
    H4 = np.linalg.matrix_power(H, 4)
    S = np.sum(H4 * H4)
    assert lam.max() ** 8 <= S * (1 + 1e-12)
    # ... and the bound is tight up to the count of values near the largest
    assert S <= n * lam.max() ** 8 * (1 + 1e-12)


@pytest.mark.parametrize("eps", [1e-4, 1e-3, 1e-2, 0.1])
@pytest.mark.parametrize("near", [1, 8, 64])
def test_never_passes_above_tau(eps, near):
    # sigma_max(R) = (1 + eps) tau with `near` singular values at it: the rule
    # must fail (a pass would drop a singular value above tau)
    rng = np.random.default_rng(12)
    m, p, tau = 256, 200, 0.37
    s = np.r_[np.full(near, (1 + eps) * tau), tau * rng.random(p - near)]
    R = with_spectrum(rng, m, p, np.sort(s)[::-1])
    assert not certificate_passes(R, tau)


@pytest.mark.parametrize("scale", [1e-6, 1.0, 1e6])
def test_passes_with_a_gap(scale):
    # the bench's situation: the rest's largest singular value about 0.7 tau,
    # a handful near it, the bulk well below (any overall scale)
    rng = np.random.default_rng(13)
    m, p = 256, 245
    tau = 0.1 * scale
    s = np.r_[0.72, 0.70, 0.69, 0.65, 0.6, 0.5 * rng.random(p - 5)] * tau
    R = with_spectrum(rng, m, p, np.sort(s)[::-1])
    assert certificate_passes(R, tau)


def test_fails_at_the_continuum_edge():
    # a random matrix whose largest singular value is 0.99 tau, with many
    # values near it: within the bound's slack, so the slice goes to the full
    # iteration (the mode's switch usually sends such slices there earlier)
    rng = np.random.default_rng(14)
    m, p = 256, 200
    R = rng.standard_normal((m, p))
    tau = np.linalg.norm(R, 2) / 0.99
    assert not certificate_passes(R, tau)
