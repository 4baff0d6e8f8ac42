"""Host logic of the hyperparameter ascent (Section 3, ADAM): the optimiser
and the learning-rate schedule, without a GPU."""
import numpy as np

from paper_2508_01864_amd import fit


def test_adam_ascends_to_the_maximum_of_a_concave_quadratic():
    c = np.array([0.7, -1.3])
    w = np.array([1.0, 30.0])
    opt = fit.Adam([3.0, 2.0])
    for j in range(4000):
        g = -2.0 * w * (opt.theta - c)
        opt.step(g, fit.learning_rate(j, 4000, 0.05, 0.001))
    assert np.max(np.abs(opt.theta - c)) <= 1e-3


def test_adam_first_step_has_the_learning_rate_size():
    # with the bias corrections, the first step is lr * g / (|g| + eps) per entry
    opt = fit.Adam([0.0, 0.0, 0.0])
    th = opt.step([5.0, -2e-3, 0.0], 0.01)
    assert np.allclose(th, [0.01, -0.01, 0.0], rtol=1e-5, atol=1e-12)


def test_learning_rate_is_linear_between_the_end_points():
    assert fit.learning_rate(0, 20000, 0.005, 0.0005) == 0.005
    assert abs(fit.learning_rate(20000, 20000, 0.005, 0.0005) - 0.0005) <= 1e-18
    assert abs(fit.learning_rate(10000, 20000, 0.005, 0.0005) - 0.00275) <= 1e-15
    assert abs(fit.learning_rate(30000, 20000, 0.005, 0.0005) - 0.0005) <= 1e-18   # clamped
