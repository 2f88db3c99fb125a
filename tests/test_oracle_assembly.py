"""Pins for the oracle's P1 assembly (Sec. 2.2): textbook stencils, exactness and invariants."""
import numpy as np
import scipy.sparse as sp

from oracle.assembly import (element_geometry, lumped_mass, stiffness,
                             stiffness_sigma_derivative)
from workloads import meshes


def test_1d_tridiagonal_stencil():
    n, L, D = 9, 1.0, 2e-3
    coords, elems = meshes.line_mesh(n, L)
    h = L / (n - 1)
    A = stiffness(coords, elems, np.full((n - 1, 1, 1), D), np.ones(n), n).toarray()
    T = (2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1))
    T[0, 0] = T[-1, -1] = 1
    assert np.allclose(A, D / h * T, rtol=1e-14, atol=0)
    ML = lumped_mass(coords, elems, n)
    ref = np.full(n, h)
    ref[[0, -1]] = h / 2
    assert np.allclose(ML, ref, rtol=1e-14)


def test_2d_isotropic_right_triangles_give_five_point_stencil():
    n, Lx = 7, 1.5
    coords, elems = meshes.square_tri_mesh(n, n, Lx, Lx)
    h = Lx / (n - 1)
    E = elems.shape[0]
    A = stiffness(coords, elems, np.broadcast_to(np.eye(2), (E, 2, 2)), np.ones(n * n), n * n).toarray()
    c = 3 * n + 3
    row = A[c]
    nz = {int(j): row[j] for j in np.nonzero(np.abs(row) > 1e-14)[0]}
    assert set(nz) == {c, c - 1, c + 1, c - n, c + n}
    assert np.isclose(nz[c], 4.0) and all(np.isclose(nz[j], -1.0) for j in nz if j != c)
    ML = lumped_mass(coords, elems, n * n)
    assert np.isclose(ML[c], h * h) and np.isclose(ML.sum(), Lx * Lx)


def _linear_energy_check(coords, elems, D, volume):
    N = coords.shape[0]
    E = elems.shape[0]
    d = coords.shape[1]
    A = stiffness(coords, elems, np.broadcast_to(D, (E, d, d)), np.ones(N), N)
    g = np.arange(1, d + 1) * 0.7
    u = coords @ g + 0.3
    assert np.isclose(u @ (A @ u), volume * g @ D @ g, rtol=1e-12)
    assert np.max(np.abs(A @ np.ones(N))) < 1e-12 * np.abs(A).max()
    assert abs(A - A.T).max() < 1e-14 * np.abs(A).max()


def test_2d_anisotropic_linear_energy():
    coords, elems = meshes.square_tri_mesh(6, 5, 2.0, 1.0)
    D = np.array([[1.2e-3, 4e-4], [4e-4, 3e-4]])
    _linear_energy_check(coords, elems, D, 2.0)


def test_3d_five_tet_mesh_is_conforming_and_exact():
    n, side = 5, 1.5
    coords, elems = meshes.cube_tet_mesh(n, side)
    vol, _ = element_geometry(coords, elems)
    h = side / (n - 1)
    assert np.isclose(vol.sum(), side ** 3)
    assert set(np.round(vol / h ** 3, 12)) == {round(1 / 6, 12), round(1 / 3, 12)}
    # conformity: every interior triangular face is shared by exactly two tets
    faces = np.sort(np.concatenate([elems[:, [0, 1, 2]], elems[:, [0, 1, 3]],
                                    elems[:, [0, 2, 3]], elems[:, [1, 2, 3]]]), axis=1)
    _, counts = np.unique(faces, axis=0, return_counts=True)
    assert counts.max() == 2
    n_boundary = 6 * 2 * (n - 1) ** 2
    assert np.sum(counts == 1) == n_boundary
    D = np.array([[1.2e-3, 1e-4, 0], [1e-4, 5e-4, 2e-4], [0, 2e-4, 3e-4]])
    _linear_energy_check(coords, elems, D, side ** 3)
    assert np.isclose(lumped_mass(coords, elems, n ** 3).sum(), side ** 3)


def test_node_sigma_mean_and_derivative():
    coords, elems = meshes.square_tri_mesh(5, 4, 1.0, 1.0)
    N, E = coords.shape[0], elems.shape[0]
    rng = np.random.default_rng(3)
    T = np.broadcast_to(np.eye(2), (E, 2, 2))
    s = rng.uniform(0.5, 2.0, N)
    ds = rng.standard_normal(N)
    A1 = stiffness(coords, elems, T, s + ds, N)
    A0 = stiffness(coords, elems, T, s, N)
    dA = stiffness_sigma_derivative(coords, elems, T, N, ds)
    # A is linear in the nodal multipliers
    assert abs((A1 - A0) - dA).max() < 1e-13
    # a constant multiplier scales the matrix
    A2 = stiffness(coords, elems, T, np.full(N, 2.5), N)
    A3 = stiffness(coords, elems, T, np.ones(N), N)
    assert abs(A2 - 2.5 * A3).max() < 1e-13
    assert sp.issparse(A0)
