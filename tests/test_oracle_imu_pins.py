"""Pins of the oracle's visual-inertial factors (oracle/imu.py): SO(3) maps
against scipy, preintegration against closed forms (constant rate, constant
acceleration, the continuous-time limit of rotation with acceleration), the
bias Jacobians against finite differences of the integration, the residual
at states built from the deltas (exactly zero), the residual Jacobians
against finite differences on the manifold, the covariance of a static IMU,
and stereo reprojection against hand-computed values.
"""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import imu


def test_so3_maps_match_scipy():
    rng = np.random.default_rng(0)
    for phi in rng.normal(size=(20, 3)):
        phi = phi * (rng.uniform(0.0, 3.0) / np.linalg.norm(phi))    # angles below pi
        R = imu.so3_exp(phi)
        np.testing.assert_allclose(R, Rotation.from_rotvec(phi).as_matrix(), atol=1e-13)
        np.testing.assert_allclose(imu.so3_log(R), phi, atol=1e-12)
    np.testing.assert_allclose(imu.so3_exp([1e-6, 0, 0]), Rotation.from_rotvec([1e-6, 0, 0]).as_matrix(),
                               atol=1e-15)


def test_right_jacobian_is_the_derivative_of_exp():
    # Exp(phi + d) = Exp(phi) Exp(Jr(phi) d) to first order
    rng = np.random.default_rng(1)
    phi = rng.normal(size=3)
    h = 1e-6
    for k in range(3):
        d = np.zeros(3)
        d[k] = h
        lhs = imu.so3_log(imu.so3_exp(phi).T @ imu.so3_exp(phi + d)) / h
        np.testing.assert_allclose(lhs, imu.right_jacobian(phi)[:, k], atol=1e-6)


def test_constant_rate_and_constant_acceleration_closed_forms():
    n, dt = 400, 0.005
    T = n * dt
    w = np.array([0.3, -0.2, 0.5])
    P = imu.preintegrate(np.tile(w, (n, 1)), np.zeros((n, 3)), dt, np.zeros(3), np.zeros(3))
    np.testing.assert_allclose(P.dR, imu.so3_exp(w * T), atol=1e-12)   # products of equal steps
    assert np.abs(P.dv).max() == 0 and np.abs(P.dp).max() == 0
    a = np.array([0.4, 1.0, -2.0])
    P = imu.preintegrate(np.zeros((n, 3)), np.tile(a, (n, 1)), dt, np.zeros(3), np.zeros(3))
    np.testing.assert_allclose(P.dv, a * T, rtol=1e-12)
    np.testing.assert_allclose(P.dp, 0.5 * a * T * T, rtol=1e-12)      # exact for the discrete sum
    assert P.dt == pytest.approx(T)


def test_rotation_with_acceleration_converges_to_the_continuous_integral():
    # dv -> int_0^T Exp(w t) a dt = T Jl(w T) a with Jl(phi) = Jr(-phi)
    w = np.array([0.0, 0.0, 1.3])
    a = np.array([1.0, 0.5, 0.0])
    T = 1.0
    errs = []
    for n in (1000, 4000):
        P = imu.preintegrate(np.tile(w, (n, 1)), np.tile(a, (n, 1)), T / n, np.zeros(3), np.zeros(3))
        want = T * imu.right_jacobian(-w * T) @ a
        errs.append(np.abs(P.dv - want).max())
    assert errs[1] < 1e-3 and errs[1] < 0.3 * errs[0]      # first-order convergence


def _trajectory_imu(seed=2, n=200, dt=0.005):
    rng = np.random.default_rng(seed)
    gyro = rng.normal(scale=0.5, size=(n, 3))
    acc = rng.normal(scale=2.0, size=(n, 3)) + np.array([0, 0, 9.81])
    return gyro, acc, dt


def test_bias_jacobians_match_finite_differences():
    gyro, acc, dt = _trajectory_imu()
    bg0, ba0 = np.array([0.01, -0.02, 0.005]), np.array([0.1, 0.0, -0.05])
    P = imu.preintegrate(gyro, acc, dt, bg0, ba0)
    h = 1e-6
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        Pg = imu.preintegrate(gyro, acc, dt, bg0 + e, ba0)
        Pa = imu.preintegrate(gyro, acc, dt, bg0, ba0 + e)
        np.testing.assert_allclose(imu.so3_log(P.dR.T @ Pg.dR) / h, P.JRg[:, k], atol=1e-5)
        np.testing.assert_allclose((Pg.dv - P.dv) / h, P.Jvg[:, k], atol=1e-5)
        np.testing.assert_allclose((Pg.dp - P.dp) / h, P.Jpg[:, k], atol=1e-5)
        np.testing.assert_allclose((Pa.dv - P.dv) / h, P.Jva[:, k], atol=1e-6)
        np.testing.assert_allclose((Pa.dp - P.dp) / h, P.Jpa[:, k], atol=1e-6)


def _states(P, seed=3, bias_offset=0.0):
    rng = np.random.default_rng(seed)
    Ri = imu.so3_exp(rng.normal(size=3))
    pi, vi = rng.normal(size=3), rng.normal(size=3)
    g, dt = imu.GRAVITY, P.dt
    Rj = Ri @ P.dR
    vj = vi + g * dt + Ri @ P.dv
    pj = pi + vi * dt + 0.5 * g * dt * dt + Ri @ P.dp
    return Ri, pi, vi, P.bg0 + bias_offset, P.ba0 + bias_offset, Rj, pj, vj


def test_residual_vanishes_at_states_built_from_the_deltas():
    gyro, acc, dt = _trajectory_imu()
    P = imu.preintegrate(gyro, acc, dt, np.array([0.01, 0.0, 0.0]), np.zeros(3))
    r = imu.inertial_residual(*_states(P), P)
    assert np.abs(np.array(r, float)).max() < 1e-12


def test_inertial_jacobian_matches_manifold_finite_differences():
    gyro, acc, dt = _trajectory_imu()
    P = imu.preintegrate(gyro, acc, dt, np.zeros(3), np.zeros(3))
    rng = np.random.default_rng(9)
    Ri, pi, vi, bgi, bai, Rj, pj, vj = _states(P, bias_offset=0.01)
    Rj = Rj @ imu.so3_exp(rng.normal(scale=0.05, size=3))      # away from zero residual
    vj = vj + rng.normal(scale=0.1, size=3)
    r0, J = imu.inertial_residual_and_jacobian(Ri, pi, vi, bgi, bai, Rj, pj, vj, P)
    h = 1e-6

    def res(d):
        x = [Ri @ imu.so3_exp(d[0:3]), pi + d[3:6], vi + d[6:9], bgi + d[9:12], bai + d[12:15],
             Rj @ imu.so3_exp(d[15:18]), pj + d[18:21], vj + d[21:24]]
        return np.array(imu.inertial_residual(*x, P), float)
    np.testing.assert_allclose(res(np.zeros(24)), r0, atol=1e-14)
    for c in range(24):
        d = np.zeros(24)
        d[c] = h
        fd = (res(d) - res(-d)) / (2 * h)
        np.testing.assert_allclose(J[:, c], fd, atol=1e-6 * max(1.0, np.abs(fd).max()))


def test_static_imu_covariance():
    # no rotation, no acceleration: the rotation block is sigma_g^2 T I and
    # the velocity block sigma_a^2 T I; symmetric positive semi-definite
    n, dt = 200, 0.005
    P = imu.preintegrate(np.zeros((n, 3)), np.zeros((n, 3)), dt, np.zeros(3), np.zeros(3),
                         sigma_g=0.01, sigma_a=0.1)
    T = n * dt
    np.testing.assert_allclose(P.cov[0:3, 0:3], 0.01 ** 2 * T * np.eye(3), rtol=1e-12)
    np.testing.assert_allclose(P.cov[3:6, 3:6], 0.1 ** 2 * T * np.eye(3), rtol=1e-12)
    assert np.linalg.eigvalsh(P.cov).min() > -1e-18


def test_stereo_reprojection_hand_values_and_jacobian():
    # camera at the origin looking down +z: Xc = X
    r = imu.stereo_residual(np.eye(3), np.zeros(3), [1.0, 2.0, 10.0], 500.0, 500.0, 320.0, 240.0,
                            0.1, [0.0, 0.0, 0.0])
    np.testing.assert_allclose(r, [370.0, 340.0, 365.0], atol=1e-12)
    rng = np.random.default_rng(4)
    R, p = imu.so3_exp(rng.normal(scale=0.3, size=3)), rng.normal(size=3)
    X = p + R @ np.array([0.5, -0.3, 8.0])
    obs = [300.0, 200.0, 290.0]
    r0, J = imu.stereo_residual_and_jacobian(R, p, X, 450.0, 460.0, 320.0, 240.0, 0.11, obs)
    h = 1e-6

    def res(d):
        return np.array(imu.stereo_residual(R @ imu.so3_exp(d[0:3]), p + d[3:6], X + d[6:9],
                                            450.0, 460.0, 320.0, 240.0, 0.11, obs), float)
    for c in range(9):
        d = np.zeros(9)
        d[c] = h
        np.testing.assert_allclose(J[:, c], (res(d) - res(-d)) / (2 * h), atol=1e-5)
