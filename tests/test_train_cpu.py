"""Host logic of the Adam driver: checkpoint and resume reproduce an
uninterrupted run.  A closed-form objective stands in for the library so the
test needs no GPU."""
import numpy as np
import torch

from paper_2107_00243_amd.train import adam_fit


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
