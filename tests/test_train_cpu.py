"""Host logic of the optimiser drivers (Adam, L-BFGS): convergence on a closed
form, checkpoint and resume.  A closed-form objective stands in for the library
so the tests need no GPU."""
import numpy as np
import torch

from paper_2107_00243_amd.train import adam_fit, lbfgs_fit


class QuadraticModel:
    """log p(theta) = -sum (log theta - c)^2 with its gradient w.r.t. theta."""

    def __init__(self, c):
        self.c = np.asarray(c, dtype=np.float64)
        self.want_stats = False
        self.last_stats = None

    def evaluate(self, theta, with_grad=True, stats=False):
        u = np.log(theta) - self.c
        logp = torch.tensor([-np.sum(u * u)])
        grad = torch.tensor(-2.0 * u / theta)
        return logp, grad


def test_adam_increases_the_objective_and_moves_towards_the_optimum():
    m = QuadraticModel([0.3, -0.2, 0.1])
    hist, theta = adam_fit(m, np.ones(3), steps=30, lr=0.05, log=lambda s: None)
    assert hist[-1]["logp"] > hist[0]["logp"]
    assert np.all(np.abs(np.log(theta) - m.c) < np.abs(m.c))


def test_checkpoint_resume_reproduces_the_uninterrupted_run(tmp_path):
    m = QuadraticModel([0.5, -0.4, 0.2, 0.0])
    th0 = np.array([1.0, 2.0, 0.5, 1.5])
    ref_hist, ref_theta = adam_fit(m, th0, steps=6, lr=0.1, log=lambda s: None)
    ck = str(tmp_path / "run.npz")
    adam_fit(m, th0, steps=3, lr=0.1, checkpoint=ck, log=lambda s: None)
    hist, theta = adam_fit(m, th0, steps=6, lr=0.1, checkpoint=ck, resume=True, log=lambda s: None)
    np.testing.assert_array_equal(theta, ref_theta)
    assert [h["logp"] for h in hist] == [h["logp"] for h in ref_hist]


class RosenbrockModel:
    """log p = -Rosenbrock(log theta_0, log theta_1): curved valley, minimum at 1, 1."""

    def __init__(self):
        self.want_stats = False
        self.last_stats = None
        self.calls = 0

    def evaluate(self, theta, with_grad=True, stats=False):
        self.calls += 1
        a, b = np.log(theta)
        f = (1 - a) ** 2 + 100 * (b - a * a) ** 2
        ga = -2 * (1 - a) - 400 * a * (b - a * a)
        gb = 200 * (b - a * a)
        return torch.tensor([-f]), torch.tensor([-ga / theta[0], -gb / theta[1]])


def test_lbfgs_solves_a_quadratic_in_a_few_iterations():
    m = QuadraticModel([0.3, -0.2, 0.1, 0.7])
    hist, theta = lbfgs_fit(m, np.ones(4), steps=20, log=lambda s: None)
    np.testing.assert_allclose(np.log(theta), m.c, atol=1e-6)
    assert len(hist) <= 6
    assert all(h2["logp"] >= h1["logp"] - 1e-12 for h1, h2 in zip(hist, hist[1:]))


def test_lbfgs_line_search_follows_a_curved_valley():
    m = RosenbrockModel()
    hist, theta = lbfgs_fit(m, np.exp([-1.2, 1.0]), steps=100, log=lambda s: None)
    np.testing.assert_allclose(np.log(theta), [1.0, 1.0], atol=1e-4)
    # every accepted iterate improves the objective (sufficient decrease)
    assert all(h2["logp"] > h1["logp"] for h1, h2 in zip(hist, hist[1:]) if h2["evaluations"] > 1)


def test_lbfgs_checkpoint_keeps_theta_and_history(tmp_path):
    m = QuadraticModel([0.5, -0.4])
    ck = str(tmp_path / "lb.npz")
    h1, th1 = lbfgs_fit(m, np.array([2.0, 0.5]), steps=2, checkpoint=ck, log=lambda s: None)
    z = np.load(ck, allow_pickle=False)
    assert int(z["step"]) == len(h1)
    np.testing.assert_array_equal(np.exp(z["log_theta"]), th1)
    h2, th2 = lbfgs_fit(m, np.array([2.0, 0.5]), steps=20, checkpoint=ck, resume=True, log=lambda s: None)
    assert h2[:len(h1)] == h1
    np.testing.assert_allclose(np.log(th2), m.c, atol=1e-6)
