"""Pins of the FP64 window-cost oracle (eq. (1) window form, Section 3.1):
gradient against central finite differences, zero cost at exact shifts,
homogeneity, and the zero-sum property of the gradient."""
import numpy as np
import pytest

from oracle import cost_f32 as cf


def _case(seed, H=12, W=15, C=3, spread=6):
    rng = np.random.default_rng(seed)
    F = [rng.standard_normal((H, W, C)) for _ in range(4)]
    hyp = np.empty((H, W, 4), np.int16)
    hyp[..., :2] = rng.integers(-spread, spread + 1, (H, W, 2))
    hyp[..., 2:] = rng.integers(0, spread + 1, (H, W, 2))
    g = rng.uniform(0.5, 1.5, (H, W))
    return F, hyp, g


@pytest.mark.parametrize("s", [1, -1])
def test_gradient_matches_central_differences(s):
    F, hyp, g = _case(1 if s > 0 else 2)
    G = cf.window_cost_grad(F, hyp, s, g)
    rng = np.random.default_rng(3)
    H, W, C = F[0].shape
    picks = [(m, int(rng.integers(H)), int(rng.integers(W)), int(rng.integers(C)))
             for m in range(4) for _ in range(6)]
    picks += [(m, 0, 0, 0) for m in range(4)] + [(m, H - 1, W - 1, C - 1) for m in range(4)]
    fdh = cf.FiniteDifferences(F, hyp, s, g)
    for (m, y, x, c) in picks:
        fd = cf.fd_grad_entry(F, hyp, s, g, m, y, x, c, eps=1e-3)
        assert abs(fd - G[m][y, x, c]) <= 1e-8 * max(1.0, abs(fd)), (m, y, x, c)
        # the bucketed helper finds the same affected pixels
        assert abs(fdh.grad_entry(m, y, x, c, eps=1e-3) - fd) <= 1e-12 * max(1.0, abs(fd))


def test_zero_cost_at_exact_shifts():
    rng = np.random.default_rng(4)
    H, W, C = 30, 40, 2
    R = rng.standard_normal((H, W, C))
    u, v, d0, d1 = 3, -2, 4, 5
    def shifted(dx, dy):
        out = np.zeros_like(R)
        yy, xx = np.indices((H, W))
        sy, sx = np.clip(yy - dy, 0, H - 1), np.clip(xx - dx, 0, W - 1)
        return R[sy, sx]
    F = [R, shifted(u, v), shifted(-d0, 0), shifted(u - d1, v)]
    hyp = np.tile(np.array([u, v, d0, d1], np.int16), (H, W, 1))
    cost = cf.window_cost(F, hyp, 1)
    inner = cost[10:20, 12:28]
    assert np.abs(inner).max() < 1e-20
    assert cost.max() > 1.0  # border pixels see clamped, different samples


def test_homogeneity_and_gradient_sum():
    F, hyp, g = _case(5, H=9, W=11, C=2)
    c1 = cf.window_cost(F, hyp, -1)
    c2 = cf.window_cost([2 * f for f in F], hyp, -1)
    assert np.allclose(c2, 4 * c1, rtol=1e-12)
    G = cf.window_cost_grad(F, hyp, -1, g)
    total = sum(x.sum() for x in G)
    assert abs(total) < 1e-9 * sum(np.abs(x).sum() for x in G)
    # Euler's theorem for a quadratic form: sum_entries F . dL/dF = 2 L
    L = (g * c1).sum()
    assert np.isclose(sum((f * gr).sum() for f, gr in zip(F, G)), 2 * L, rtol=1e-10)
