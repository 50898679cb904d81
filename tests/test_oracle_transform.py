"""Pins of the control right-transformation (oracle/transform.py): the paper's
repeat-the-column choice T = [1 ... 1] reduces the reconstruction to the column mean,
the reconstruction is a left inverse of the expansion, a square invertible T gives
U T^{-1}, and the result is the least-squares solution of u T = U."""
import numpy as np

from oracle import transform as tr


def test_ones_row_gives_column_mean():
    rng = np.random.default_rng(0)
    U = rng.standard_normal((5, 7))
    u = tr.project(U, np.ones((1, 7)))
    assert np.allclose(u, U.mean(axis=1, keepdims=True), atol=1e-14)


def test_projection_is_a_left_inverse_of_the_expansion():
    rng = np.random.default_rng(1)
    T = rng.standard_normal((3, 9))
    u = rng.standard_normal((4, 3))
    assert np.allclose(tr.project(tr.expand(u, T), T), u, atol=1e-12)


def test_square_invertible_transform():
    rng = np.random.default_rng(2)
    T = rng.standard_normal((6, 6)) + 3 * np.eye(6)
    U = rng.standard_normal((2, 6))
    assert np.allclose(tr.project(U, T), U @ np.linalg.inv(T), atol=1e-12)


def test_least_squares_optimality():
    # u minimises ||u T - U||_F: the residual is orthogonal to the row space of T
    rng = np.random.default_rng(3)
    T = rng.standard_normal((2, 8))
    U = rng.standard_normal((3, 8))
    u = tr.project(U, T)
    assert np.allclose((u @ T - U) @ T.T, 0.0, atol=1e-12)
    assert np.allclose(u, np.linalg.lstsq(T.T, U.T, rcond=None)[0].T, atol=1e-12)
