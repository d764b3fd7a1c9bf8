"""Checks of the seeded input generators (no solver involved)."""
import numpy as np
import scipy.linalg

from paper_2601_14414_amd import workloads as W


def test_zoh_matches_quadrature():
    """ZOH: A_d = exp(A_c dt), B_d = int_0^dt exp(A_c s) ds B_c (Simpson)."""
    Ac, Bc = W.mass_spring_continuous(4)
    Ad, Bd = W.mass_spring(4)
    np.testing.assert_allclose(Ad, scipy.linalg.expm(Ac * 0.1), atol=1e-13)
    ss = np.linspace(0.0, 0.1, 401)
    vals = np.array([scipy.linalg.expm(Ac * s) @ Bc for s in ss])
    h = ss[1] - ss[0]
    simpson = h / 3 * (vals[0] + vals[-1] + 4 * vals[1:-1:2].sum(0) + 2 * vals[2:-1:2].sum(0))
    np.testing.assert_allclose(Bd, simpson, atol=1e-12)


def test_mass_spring_shapes_and_stability():
    for p in (4, 12):
        A, B = W.mass_spring(p)
        assert A.shape == (2 * p, 2 * p) and B.shape == (2 * p, p - 1)
        rad = np.max(np.abs(np.linalg.eigvals(A)))
        assert 0.99 < rad < 1.0  # damped, lightly


def test_random_batch_recipe():
    ps = W.random_batch(64, base_seed=5)
    for p in ps:
        assert p.nx in (4, 8, 12, 16) and p.nu in (1, 2, 3, 4) and 32 <= p.N <= 512
        sv = np.linalg.svd(p.A, compute_uv=False)
        assert np.all(sv >= 0.95 - 1e-12) and np.all(sv <= 1.05 + 1e-12)
        assert np.all(np.abs(p.x0) <= 1.0)
    # determinism
    q = W.random_batch_instance(5 + 3)
    np.testing.assert_array_equal(q.A, ps[3].A)


def test_cartpole_energy_and_jacobians():
    """The plant conserves energy (frictionless, u = 0) and the complex-step
    Jacobians agree with central differences."""
    M, m, l, g = 1.0, 0.1, 0.5, 9.81

    def energy(x):
        p, pd, th, thd = x
        return (0.5 * (M + m) * pd ** 2 + m * l * pd * thd * np.cos(th)
                + 0.5 * (4.0 / 3.0) * m * l * l * thd ** 2 + m * g * l * np.cos(th))

    x = np.array([0.0, 0.3, 2.5, 0.7])
    e0 = energy(x)
    for _ in range(500):
        x = W.cartpole_rk4(x, np.zeros(1), dt=0.002, substeps=1)
    assert abs(energy(x) - e0) < 1e-10
    x = np.array([0.1, -0.2, 2.0, 0.4])
    u = np.array([1.5])
    A, B = W.cartpole_jacobians(x, u)
    h = 1e-6
    for j in range(4):
        d = np.zeros(4); d[j] = h
        fd = (W.cartpole_fd(x + d, u) - W.cartpole_fd(x - d, u)) / (2 * h)
        np.testing.assert_allclose(A[:, j], fd, atol=1e-8)
    fd = (W.cartpole_fd(x, u + h) - W.cartpole_fd(x, u - h)) / (2 * h)
    np.testing.assert_allclose(B[:, 0], fd, atol=1e-8)


def test_cartpole_linearization_affine_term():
    xs = np.random.default_rng(0).uniform(-1, 1, (5, 4))
    us = np.random.default_rng(1).uniform(-1, 1, (5, 1))
    A, B, e = W.cartpole_linearize(xs, us)
    for k in range(5):
        np.testing.assert_allclose(A[k] @ xs[k] + B[k] @ us[k] + e[k], W.cartpole_fd(xs[k], us[k]),
                                   atol=1e-13)
        # all stages at once give the single-point complex-step Jacobians
        Ak, Bk = W.cartpole_jacobians(xs[k], us[k])
        np.testing.assert_allclose(A[k], Ak, rtol=0, atol=1e-15)
        np.testing.assert_allclose(B[k], Bk, rtol=0, atol=1e-15)


def test_rti_shift():
    N, nx = 6, 4
    pred = np.arange(N * 5, dtype=float).reshape(N, 5)
    xs, us = W.rti_shift(np.array([9.0, 9, 9, 9]), pred)
    np.testing.assert_array_equal(xs[0], [9, 9, 9, 9])
    np.testing.assert_array_equal(xs[2], pred[2][:nx])
    np.testing.assert_array_equal(us[0], pred[1][nx:])
    np.testing.assert_array_equal(us[N - 1], pred[N - 1][nx:])


def test_pack_offsets():
    ps = W.random_batch(8, base_seed=11)
    pk = W.pack(ps)
    assert pk.A.size == sum(p.nx * p.nx for p in ps)
    assert pk.x0.size == sum(p.nx for p in ps)
    assert pk.time_varying == 0
