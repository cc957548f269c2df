"""Pins of the CPU oracle's thermal stencils against closed forms and brute force.

The update (2D, per step, neighbour indices clamped to the grid):
    T' = T + c*(P + (Tn+Ts-2T)/Ry + (Te+Tw-2T)/Rx + (Tamb-T)/Rz)
and in 3D the extra term (Tu+Td-2T)/Rz.  The clamped second difference in
one direction equals minus the Laplacian of a path graph, so the whole step
is the affine map  T' = M T + q  with
    M = I - c*(L_y (x) I / Ry + I (x) L_x / Rx + I / Rz),  q = c*(P + Tamb/Rz).
The DCT-II vectors cos(pi k (i+1/2) / N) are the eigenvectors of L_path with
eigenvalues 4 sin^2(pi k / 2N); the Laplacian's rows sum to zero, so the mean
obeys a scalar recurrence.  None of these uses the oracle's own code.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth


def path_laplacian(n):
    L = [[Fraction(0)] * n for _ in range(n)]
    for i in range(n):
        for j in (i - 1, i + 1):
            if 0 <= j < n:
                L[i][i] += 1
                L[i][j] -= 1
    return L


def kron(A, B):
    na, nb = len(A), len(B)
    return [[A[i // nb][j // nb] * B[i % nb][j % nb] for j in range(na * nb)] for i in range(na * nb)]


def eye(n):
    return [[Fraction(int(i == j)) for j in range(n)] for i in range(n)]


def affine_operator_2d(ny, nx, c, Rx, Ry, Rz):
    Ly = kron(path_laplacian(ny), eye(nx))
    Lx = kron(eye(ny), path_laplacian(nx))
    n = ny * nx
    return [[(1 if i == j else 0) - c * (Ly[i][j] / Ry + Lx[i][j] / Rx + (1 if i == j else 0) / Rz)
             for j in range(n)] for i in range(n)]


def affine_operator_3d(nz, ny, nx, c, Rx, Ry, Rz):
    Lz = kron(kron(path_laplacian(nz), eye(ny)), eye(nx))
    Ly = kron(kron(eye(nz), path_laplacian(ny)), eye(nx))
    Lx = kron(kron(eye(nz), eye(ny)), path_laplacian(nx))
    n = nz * ny * nx
    return [[(1 if i == j else 0) - c * (Lz[i][j] / Rz + Ly[i][j] / Ry + Lx[i][j] / Rx + (1 if i == j else 0) / Rz)
             for j in range(n)] for i in range(n)]


def matvec(M, v):
    return [sum((a * b for a, b in zip(row, v) if a), Fraction(0)) for row in M]


def exact(x):
    return [Fraction(float(v)) for v in np.ravel(x)]


C, RX, RY, RZ, TAMB = Fraction(1, 1000), Fraction(1), Fraction(2), Fraction(10), Fraction(300)
KW = dict(c=1e-3, Rx=1.0, Ry=2.0, Rz=10.0, Tamb=300.0)


@pytest.mark.parametrize("ny,nx", [(8, 8), (5, 7)])
def test_heat2d_brute_force_exact_rationals(ny, nx):
    T0, P = synth.heat2d_init(1, ny, nx)
    M = affine_operator_2d(ny, nx, C, RX, RY, RZ)
    q = [C * (p + TAMB / RZ) for p in exact(P)]
    t = exact(T0)
    for n in range(1, 11):
        t = [a + b for a, b in zip(matvec(M, t), q)]
        got = oracle.heat2d(T0, P, n, **KW).ravel()
        ref = np.array([float(v) for v in t])
        assert np.max(np.abs(got - ref)) / np.max(np.abs(ref)) < 1e-14


def test_heat2d_brute_force_long_run_float64():
    ny, nx = 8, 8
    T0, P = synth.heat2d_init(2, ny, nx)
    M = np.array([[float(v) for v in row] for row in affine_operator_2d(ny, nx, C, RX, RY, RZ)])
    q = 1e-3 * (P.astype(np.float64).ravel() + 300.0 / 10.0)
    # T_n = M^n T0 + (I - M)^{-1} (I - M^n) q
    Mn = np.linalg.matrix_power(M, 1000)
    ref = Mn @ T0.astype(np.float64).ravel() + np.linalg.solve(np.eye(64) - M, (np.eye(64) - Mn) @ q)
    got = oracle.heat2d(T0, P, 1000, **KW).ravel()
    assert np.max(np.abs(got - ref)) / np.max(np.abs(ref)) < 1e-12


@pytest.mark.parametrize("k,l", [(0, 0), (3, 2), (1, 0), (0, 4), (11, 9)])
def test_heat2d_single_dct_mode_decay(k, l):
    ny, nx, A, p, n = 12, 10, 5.0, 0.25, 400
    i = np.arange(ny)[:, None]
    j = np.arange(nx)[None, :]
    phi = np.cos(np.pi * k * (i + 0.5) / ny) * np.cos(np.pi * l * (j + 0.5) / nx)
    teq = 300.0 + p * 10.0
    T0 = teq + A * phi
    P = np.full((ny, nx), p)
    g = 1 - 1e-3 * (4 * np.sin(np.pi * k / (2 * ny)) ** 2 / 2.0 + 4 * np.sin(np.pi * l / (2 * nx)) ** 2 / 1.0 + 1 / 10.0)
    got = oracle.heat2d(T0, P, n, **KW)
    ref = teq + A * g ** n * phi
    assert np.max(np.abs(got - ref)) < 1e-11 * A


def test_heat2d_mean_recurrence():
    ny, nx, n = 40, 24, 1000
    T0, P = synth.heat2d_init(3, ny, nx)
    m0 = np.mean(T0.astype(np.float64))
    pbar = np.mean(P.astype(np.float64))
    c, Rz, Tamb = 1e-3, 10.0, 300.0
    ref = Tamb + pbar * Rz + (m0 - Tamb - pbar * Rz) * (1 - c / Rz) ** n
    got = np.mean(oracle.heat2d(T0, P, n, **KW))
    assert abs(got - ref) / ref < 1e-13


def test_heat2d_transpose_symmetry():
    T0, P = synth.heat2d_init(4, 9, 13)
    kw = dict(KW, Ry=1.0)
    a = oracle.heat2d(T0, P, 50, **kw)
    b = oracle.heat2d(T0.T, P.T, 50, **kw)
    assert np.max(np.abs(a - b.T)) < 1e-12


def test_heat2d_float32_close_to_float64():
    # The float32 instantiation follows the same formula; on the 256x256,
    # 1000-step workload it stays within a few float32 ulps of 330 K.
    T0, P = synth.heat2d_init(0, 256, 256)
    a = oracle.heat2d(T0, P, 1000, dtype=np.float32)
    b = oracle.heat2d(T0, P, 1000)
    assert np.max(np.abs(a - b)) / np.max(np.abs(b)) < 2e-5


def test_heat3d_brute_force_exact_rationals():
    nz, ny, nx = 3, 4, 5
    T0, P2 = synth.heat3d_init(5, nz, ny, nx)
    P = np.zeros((nz, ny, nx), np.float32)
    P[0] = P2
    M = affine_operator_3d(nz, ny, nx, C, RX, RY, RZ)
    q = [C * (p + TAMB / RZ) for p in exact(P)]
    t = exact(T0)
    for n in range(1, 8):
        t = [a + b for a, b in zip(matvec(M, t), q)]
        got = oracle.heat3d(T0, P2, n, **KW).ravel()
        ref = np.array([float(v) for v in t])
        assert np.max(np.abs(got - ref)) / np.max(np.abs(ref)) < 1e-14


@pytest.mark.parametrize("m,k,l", [(1, 2, 3), (2, 0, 1), (0, 0, 0), (3, 5, 4)])
def test_heat3d_single_dct_mode_decay(m, k, l):
    nz, ny, nx, A, p, n = 4, 6, 5, 3.0, 0.5, 300
    z = np.arange(nz)[:, None, None]
    i = np.arange(ny)[None, :, None]
    j = np.arange(nx)[None, None, :]
    phi = (np.cos(np.pi * m * (z + 0.5) / nz) * np.cos(np.pi * k * (i + 0.5) / ny)
           * np.cos(np.pi * l * (j + 0.5) / nx))
    teq = 300.0 + p * 10.0
    T0 = teq + A * phi
    P = np.full((nz, ny, nx), p)
    g = 1 - 1e-3 * (4 * np.sin(np.pi * m / (2 * nz)) ** 2 / 10.0 + 4 * np.sin(np.pi * k / (2 * ny)) ** 2 / 2.0
                    + 4 * np.sin(np.pi * l / (2 * nx)) ** 2 / 1.0 + 1 / 10.0)
    got = oracle.heat3d(T0, P, n, **KW)
    assert np.max(np.abs(got - (teq + A * g ** n * phi))) < 1e-11 * A


def test_heat3d_mean_recurrence_power_in_bottom_layer():
    nz, ny, nx, n = 8, 16, 12, 2000
    T0, P2 = synth.heat3d_init(6, nz, ny, nx)
    m0 = np.mean(T0.astype(np.float64))
    pbar = np.sum(P2.astype(np.float64)) / (nz * ny * nx)   # zero above layer 0
    ref = 300.0 + pbar * 10.0 + (m0 - 300.0 - pbar * 10.0) * (1 - 1e-3 / 10.0) ** n
    got = np.mean(oracle.heat3d(T0, P2, n, **KW))
    assert abs(got - ref) / ref < 1e-13
