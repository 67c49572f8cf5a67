"""The nebula search's CMA-ES sampler (host logic): convergence on textbook
objectives, optimum on the boundary of the box, and determinism by seed."""
import numpy as np

from paper_2104_12922_amd.cmaes import CMAES
from paper_2104_12922_amd.nebula import with_curves


def _minimise(f, es, evals):
    best = np.inf
    done = 0
    while done < evals:
        X = es.ask()
        v = [f(x) for x in X]
        es.tell(v)
        best = min(best, min(v))
        done += len(v)
    return best


def test_sphere_and_ellipsoid_converge():
    n = 10
    es = CMAES(np.full(n, 3.0), 1.0, -5.0, 5.0, seed=1)
    assert _minimise(lambda x: float(np.sum(x ** 2)), es, 3000) < 1e-10
    # ill-conditioned ellipsoid (condition 1e4): needs the covariance update
    scale = 10.0 ** (2.0 * np.arange(n) / (n - 1))
    es = CMAES(np.full(n, 2.0), 1.0, -5.0, 5.0, seed=2)
    assert _minimise(lambda x: float(np.sum((scale * x) ** 2)), es, 8000) < 1e-8


def test_rosenbrock():
    n = 5
    f = lambda x: float(np.sum(100.0 * (x[1:] - x[:-1] ** 2) ** 2 + (1.0 - x[:-1]) ** 2))
    es = CMAES(np.zeros(n), 0.5, -3.0, 3.0, seed=3)
    assert _minimise(f, es, 12000) < 1e-8


def test_box_optimum_on_the_boundary():
    # minimum of sum (x - 2)^2 over [-1, 1]^4 is the corner x = 1
    es = CMAES(np.zeros(4), 0.5, -1.0, 1.0, seed=4)
    best = _minimise(lambda x: float(np.sum((x - 2.0) ** 2)), es, 2000)
    assert best < 4.0 + 1e-8
    assert np.allclose(es.mean, 1.0, atol=1e-4)
    X = es.ask()
    assert np.all(X <= 1.0) and np.all(X >= -1.0)


def test_fold_is_the_reflection_into_the_box():
    es = CMAES(np.zeros(1), 0.5, -1.0, 1.0)
    x = np.array([-1.0, -0.3, 0.0, 0.7, 1.0, 1.25, 2.5, 3.0, -1.5, -3.2, 5.0])
    want = np.array([-1.0, -0.3, 0.0, 0.7, 1.0, 0.75, -0.5, -1.0, -0.5, 0.8, 1.0])
    assert np.allclose(es.fold(x), want, atol=1e-15)


def test_default_parameters_and_determinism():
    es = CMAES(np.zeros(78), 0.3, -1.0, 1.0, seed=5)
    assert es.lam == 4 + int(3 * np.log(78)) == 17 and es.mu == 8
    assert abs(es.w.sum() - 1.0) < 1e-15 and np.all(np.diff(es.w) < 0)
    a = CMAES(np.zeros(6), 0.3, -1.0, 1.0, seed=9)
    b = CMAES(np.zeros(6), 0.3, -1.0, 1.0, seed=9)
    for _ in range(3):
        xa, xb = a.ask(), b.ask()
        assert np.array_equal(xa, xb)
        v = [float(np.sum(x ** 2)) for x in xa]
        a.tell(v)
        b.tell(v)


def test_with_curves():
    tab = np.arange(78 * 4, dtype=np.float64).reshape(78, 4)
    out = with_curves(tab, [0, 5], [-1.0, 1.0])
    assert out[0, 2] == 0.1 and out[5, 2] == 10.0
    keep = np.ones(78, dtype=bool)
    keep[[0, 5]] = False
    assert np.array_equal(out[keep], tab[keep]) and np.array_equal(out[:, [0, 1, 3]], tab[:, [0, 1, 3]])
    assert tab[0, 2] == 2.0           # the input is not modified
