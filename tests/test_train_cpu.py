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


# ------------------------------------------------- validation early stopping

def _path_loss(c_val):
    """Validation loss |log theta - c_val|^2: minimised off the training optimum,
    so the iterates pass its minimum and the loss rises again."""
    c_val = np.asarray(c_val, dtype=np.float64)
    calls = []

    def validate(theta):
        calls.append(np.array(theta))
        u = np.log(theta) - c_val
        return float(np.sum(u * u))
    return validate, calls


def _check_early_stop(hist, theta, validate_calls, theta0, patience, vloss):
    losses = [vloss(theta0)] + [h["validation"] for h in hist]
    best = int(np.argmin(losses))
    # the theta returned is the one of lowest validation loss ...
    np.testing.assert_array_equal(theta, theta0 if best == 0 else hist[best - 1]["theta"])
    # ... and the run went on exactly `patience` steps past it
    assert len(hist) == best + patience
    assert all(losses[i] >= losses[best] for i in range(best + 1, len(losses)))
    assert len(validate_calls) == len(losses)


def test_lbfgs_early_stopping_returns_the_best_validation_theta():
    m = RosenbrockModel()
    th0 = np.exp([-1.2, 1.0])
    validate, calls = _path_loss([0.0, -0.3])
    for patience in (1, 3):
        calls.clear()
        hist, theta = lbfgs_fit(m, th0, steps=100, log=lambda s: None, validate=validate, patience=patience)
        _check_early_stop(hist, theta, calls, th0, patience, lambda t: float(np.sum((np.log(t) - [0.0, -0.3]) ** 2)))
        assert len(hist) < 100


def test_adam_early_stopping_returns_the_best_validation_theta():
    m = QuadraticModel([1.0, -1.0])
    th0 = np.ones(2)
    validate, calls = _path_loss([0.4, -0.2])
    hist, theta = adam_fit(m, th0, steps=200, lr=0.05, log=lambda s: None, validate=validate, patience=2)
    _check_early_stop(hist, theta, calls, th0, 2, lambda t: float(np.sum((np.log(t) - [0.4, -0.2]) ** 2)))
    assert 2 < len(hist) < 200


def test_early_stopping_without_improvement_keeps_the_start():
    m = QuadraticModel([1.0, 1.0])
    th0 = np.ones(2)
    validate, calls = _path_loss([-0.5, -0.5])      # every step moves away from it
    hist, theta = lbfgs_fit(m, th0, steps=20, log=lambda s: None, validate=validate, patience=2)
    np.testing.assert_array_equal(theta, th0)
    assert len(hist) == 2


def test_early_stopping_checkpoint_resume_matches_the_uninterrupted_run(tmp_path):
    import pytest
    m = QuadraticModel([1.0, -1.0, 0.5])
    th0 = np.ones(3)
    validate, _ = _path_loss([0.5, -0.4, 0.1])
    ref_hist, ref_theta = adam_fit(m, th0, steps=200, lr=0.05, log=lambda s: None, validate=validate, patience=3)
    cut = len(ref_hist) - 2
    ck = str(tmp_path / "es.npz")
    adam_fit(m, th0, steps=cut, lr=0.05, checkpoint=ck, log=lambda s: None, validate=validate, patience=3)
    hist, theta = adam_fit(m, th0, steps=200, lr=0.05, checkpoint=ck, resume=True, log=lambda s: None,
                           validate=validate, patience=3)
    np.testing.assert_array_equal(theta, ref_theta)
    assert [h["validation"] for h in hist] == [h["validation"] for h in ref_hist]
    with pytest.raises(ValueError):
        adam_fit(m, th0, steps=2, validate=validate, patience=0, log=lambda s: None)


def test_validation_scores_against_library_densities():
    from scipy.stats import norm
    from paper_2107_00243_amd.model import validation_score

    class Fixed:
        def predict(self, theta, Xstar, with_var=False):
            mean = np.linspace(-1.0, 1.0, len(Xstar))
            return mean, (np.full(len(Xstar), 0.3) if with_var else None)

    rng = np.random.default_rng(3)
    Xv, yv = rng.normal(size=(9, 2)), rng.normal(size=9)
    theta = np.array([1.0, 2.0, 0.2])                 # sigma^2 = 0.2 adds to the latent 0.3
    mean = np.linspace(-1.0, 1.0, 9)
    assert abs(validation_score(Fixed(), Xv, yv, "rmse")(theta) - np.sqrt(np.mean((mean - yv) ** 2))) < 1e-15
    nll = -np.mean(norm.logpdf(yv, loc=mean, scale=np.sqrt(0.5)))
    assert abs(validation_score(Fixed(), Xv, yv, "nll")(theta) - nll) < 1e-13


def test_split_validation_is_a_seeded_partition():
    from paper_2107_00243_amd.train import split_validation
    X = np.arange(40.0).reshape(20, 2)
    y = np.arange(20.0)
    Xt, yt, Xv, yv = split_validation(X, y, 0.25, seed=5)
    assert len(yv) == 5 and len(yt) == 15
    assert sorted(np.concatenate([yt, yv]).tolist()) == y.tolist()
    np.testing.assert_array_equal(Xt[:, 1], 2 * yt + 1)
    Xt2, yt2, Xv2, yv2 = split_validation(X, y, 0.25, seed=5)
    np.testing.assert_array_equal(yv, yv2)
