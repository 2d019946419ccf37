"""Pins of the periodic Anderson extrapolation oracle (Section 3.3): the
plain damped step, the least-squares property of the correction, a library
solve, and the acceleration of a linear fixed-point iteration."""
import numpy as np

from oracle import pae


def test_before_start_and_plain_steps():
    rng = np.random.default_rng(0)
    m = 50
    act = np.ones(m, bool)
    act[:5] = False
    P = pae.PAE(m, mr=4, q=4, q0=10, alpha=0.9, xi=1.0)
    x0, x1 = rng.uniform(0.2, 0.8, m), rng.uniform(0.2, 0.8, m)
    out, used = P.step(x0, x1, act, 9)                  # before q0: unchanged
    assert used == 0 and np.array_equal(out, x1)
    out, used = P.step(x0, x1, act, 10)                 # it = 0: mix = xi = 1 -> the OC design
    assert used == 0 and np.allclose(out[act], x1[act]) and np.array_equal(out[~act], x1[~act])
    x2, x3 = rng.uniform(0.2, 0.8, m), rng.uniform(0.2, 0.8, m)
    out, used = P.step(x2, x3, act, 11)                 # it = 1: mix = alpha, no history yet
    assert used == 0 and np.allclose(out[act], x2[act] + 0.9 * (x3 - x2)[act])


def test_correction_is_the_least_squares_solution():
    rng = np.random.default_rng(1)
    m = 200
    act = np.ones(m, bool)
    P = pae.PAE(m, mr=4, q=4, q0=0, alpha=0.9, xi=1.0)
    xs = [rng.uniform(0.3, 0.7, m)]
    uses = []
    for loop in range(0, 10):
        x_post = np.clip(xs[-1] + 0.05 * rng.standard_normal(m), 0, 1)
        out, used = P.step(xs[-1], x_post, act, loop)
        uses.append(used)
        if used:
            r = x_post - xs[-1]
            R, X = P.R[:, :used], P.X[:, :used]
            g = np.linalg.lstsq(R, r, rcond=None)[0]
            mix = 0.9
            want = np.clip(xs[-1] + mix * r - (X + mix * R) @ g, 0, 1)
            assert np.allclose(out, want, atol=1e-10)
        xs.append(out)
    # with q0 = 0 the step counter is it = loop; corrections at it > 1 with
    # (it - 1) mod q = 0, i.e. it = 5 and 9, each with min(it, m_r) = 4
    # history columns (written at it = 2, 3, 4, 5 and then 6 .. 9)
    assert uses == [0, 0, 0, 0, 0, 4, 0, 0, 0, 4]


def test_solve_pivot_matches_library_and_handles_singular():
    rng = np.random.default_rng(2)
    for n in (1, 2, 3, 4):
        A = rng.standard_normal((n, n)) + n * np.eye(n)
        b = rng.standard_normal(n)
        assert np.allclose(pae.solve_pivot(A, b), np.linalg.solve(A, b), atol=1e-12)
    A = np.array([[1.0, 0.0], [0.0, 0.0]])
    assert np.allclose(pae.solve_pivot(A, np.array([2.0, 3.0])), [2.0, 0.0])


def test_accelerates_a_linear_fixed_point_iteration():
    rng = np.random.default_rng(3)
    m = 40
    Q = np.linalg.qr(rng.standard_normal((m, m)))[0]
    A = Q @ np.diag(np.linspace(0.2, 0.97, m)) @ Q.T
    xstar = rng.uniform(0.3, 0.7, m)            # the fixed point, inside the box
    b = xstar - A @ xstar
    U = lambda x: A @ x + b
    act = np.ones(m, bool)

    def run(accel, iters=40):
        x = np.full(m, 0.3)
        P = pae.PAE(m, mr=4, q=4, q0=0 if accel else 10 ** 9, alpha=1.0, xi=1.0)
        for loop in range(iters):
            x, _ = P.step(x, U(x), act, loop)
        return np.linalg.norm(x - xstar)

    assert run(True) < 1e-3 * run(False)


def test_early_correction_uses_every_written_column():
    """q < m_r: the first correction (it = 3) uses the two differences formed
    at it = 2 and it = 3 (the code's history has grown to three columns, the
    first still zero and dropping out), i.e. the least-squares fit over those
    two columns only."""
    rng = np.random.default_rng(4)
    m = 120
    act = np.ones(m, bool)
    P = pae.PAE(m, mr=4, q=2, q0=0, alpha=0.8, xi=0.7)
    x = rng.uniform(0.3, 0.7, m)
    pres, rs = [], []
    for loop in range(4):
        x_post = np.clip(x + 0.05 * rng.standard_normal(m), 0, 1)
        pres.append(x.copy())
        rs.append(x_post - x)
        out, used = P.step(x, x_post, act, loop)
        if loop == 3:
            assert used == 3
            Xc = np.stack([pres[2] - pres[1], pres[3] - pres[2]], 1)
            Rc = np.stack([rs[2] - rs[1], rs[3] - rs[2]], 1)
            g = np.linalg.lstsq(Rc, rs[3], rcond=None)[0]
            mix = 0.8                               # it = 3 is not a multiple of q
            want = np.clip(pres[3] + mix * rs[3] - (Xc + mix * Rc) @ g, 0, 1)
            assert np.allclose(out, want, atol=1e-10)
        else:
            assert used == 0
        x = out
