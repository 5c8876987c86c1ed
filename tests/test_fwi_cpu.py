"""Host logic of the FWI loop (eq. 7): the batched optimiser on objectives
with known minimisers (CPU tensors, no library call)."""
import numpy as np
import pytest
import torch

from paper_2603_04070_amd.fwi import lbfgs_direction, minimize


def _quadratic(seed, shapes, cond=1e3):
    rng = np.random.default_rng(seed)
    W = [torch.from_numpy(np.exp(rng.uniform(0, np.log(cond), s))) for s in shapes]
    X = [torch.from_numpy(rng.uniform(1450, 1650, s)) for s in shapes]

    def f(xs):
        return [float((w * (x - t) ** 2).sum()) for w, x, t in zip(W, xs, X)]

    def fg(xs):
        return f(xs), [2 * w * (x - t) for w, x, t in zip(W, xs, X)]
    return f, fg, X


def test_lbfgs_direction_matches_dense_bfgs():
    """The two-loop recursion equals -H g for the inverse-Hessian estimate
    built explicitly by the BFGS update from H0 = (s.y / y.y) I, and
    satisfies the secant condition H y_k = s_k of the newest pair."""
    rng = np.random.default_rng(1)
    n = 8
    M = rng.standard_normal((n, n))
    A = torch.from_numpy(M @ M.T + n * np.eye(n))
    S = [torch.from_numpy(rng.standard_normal(n)) for _ in range(4)]
    Y = [A @ s for s in S]
    g = torch.from_numpy(rng.standard_normal(n))
    eye = torch.eye(n, dtype=torch.float64)
    H = float(S[-1] @ Y[-1] / (Y[-1] @ Y[-1])) * eye
    for s, y in zip(S, Y):
        r = 1.0 / float(y @ s)
        H = (eye - r * torch.outer(s, y)) @ H @ (eye - r * torch.outer(y, s)) + r * torch.outer(s, s)
    assert torch.allclose(lbfgs_direction(g, S, Y), -H @ g, rtol=1e-10, atol=1e-12)
    assert torch.allclose(lbfgs_direction(Y[-1], S, Y), -S[-1], rtol=1e-10, atol=1e-12)


def test_lbfgs_direction_without_pairs_is_steepest_descent():
    g = torch.tensor([1.0, -2.0, 3.0], dtype=torch.float64)
    assert torch.equal(lbfgs_direction(g, [], []), -g)


def test_minimize_batched_quadratics():
    """Both methods never increase the misfit; on quadratics of condition
    1e3 L-BFGS(5) gains over three orders of magnitude in 40 steps and beats
    steepest descent by far."""
    f, fg, X = _quadratic(3, [(7, 5), (4, 9)])
    x0 = [torch.full_like(t, 1500.0) for t in X]
    final = {}
    for method in ("lbfgs", "descent"):
        xs, hist = minimize(fg, f, x0, 40, method=method, step=20.0)
        for i in range(2):
            Js = [h[i] for h in hist]
            assert all(b <= a for a, b in zip(Js, Js[1:])), "misfit must never increase"
        final[method] = [hist[-1][i] / hist[0][i] for i in range(2)]
    assert max(final["lbfgs"]) <= 1e-3
    assert all(a * 10 <= b for a, b in zip(final["lbfgs"], final["descent"]))


def test_minimize_respects_bounds():
    f, fg, X = _quadratic(4, [(6, 6)], cond=10.0)
    lo, hi = 1500.0, 1600.0
    x0 = [torch.full_like(X[0], 1550.0)]
    xs, hist = minimize(fg, f, x0, 60, method="lbfgs", step=20.0, lo=lo, hi=hi)
    assert float(xs[0].min()) >= lo and float(xs[0].max()) <= hi
    # the bound-constrained minimiser of a separable quadratic is the clamp
    assert torch.allclose(xs[0], X[0].clamp(lo, hi), atol=0.5)


def test_minimize_per_channel_bounds():
    """Tensor bounds broadcast per channel (the joint c / rho inversion)."""
    f, fg, X = _quadratic(5, [(2, 5, 5)], cond=10.0)
    lo = torch.tensor([1500.0, 1520.0], dtype=torch.float64).view(2, 1, 1)
    hi = torch.tensor([1600.0, 1560.0], dtype=torch.float64).view(2, 1, 1)
    x0 = [torch.full_like(X[0], 1540.0)]
    xs, hist = minimize(fg, f, x0, 60, method="lbfgs", step=20.0, lo=lo, hi=hi)
    assert torch.all(xs[0] >= lo) and torch.all(xs[0] <= hi)
    assert torch.allclose(xs[0], torch.max(torch.min(X[0], hi), lo), atol=0.5)
