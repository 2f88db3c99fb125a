"""Structured simplicial meshes and seeded coefficient fields.

Input data only: coordinates, element connectivity, per-element unit
conductivity tensors and per-node conductivity multipliers.  No finite-element
arithmetic (volumes, gradients, matrices) happens here; the oracle and the
library assemble independently from these arrays.
"""
import numpy as np
from scipy.ndimage import gaussian_filter


def line_mesh(n, length):
    """n uniform nodes on [0, length]; elements are the n-1 segments."""
    coords = np.linspace(0.0, length, n).reshape(n, 1)
    i = np.arange(n - 1, dtype=np.int32)
    elems = np.stack([i, i + 1], axis=1)
    return coords, elems


def square_tri_mesh(nx, ny, lx, ly):
    """nx*ny grid nodes on [0,lx]x[0,ly]; each cell split along its (i,j)-(i+1,j+1) diagonal.

    Node (i, j) (i along x) has id j*nx + i.  Element order: cell-major
    (cell (i, j) at index j*(nx-1) + i), two triangles per cell.
    """
    x = np.linspace(0.0, lx, nx)
    y = np.linspace(0.0, ly, ny)
    X, Y = np.meshgrid(x, y, indexing="xy")
    coords = np.stack([X.ravel(), Y.ravel()], axis=1)
    jj, ii = np.meshgrid(np.arange(ny - 1), np.arange(nx - 1), indexing="ij")
    n00 = (jj * nx + ii).ravel()
    n10 = n00 + 1
    n01 = n00 + nx
    n11 = n01 + 1
    t1 = np.stack([n00, n10, n11], axis=1)
    t2 = np.stack([n00, n11, n01], axis=1)
    elems = np.stack([t1, t2], axis=1).reshape(-1, 3).astype(np.int32)
    return coords, elems


def cube_tet_mesh(n, side):
    """n^3 grid nodes on [0, side]^3, 5 tetrahedra per hexahedron.

    The central tetrahedron of each hexahedron joins its four corners whose
    global index parity (I+J+K) is even, so every face diagonal joins two even
    vertices and the mesh is conforming.  Node (i, j, k) has id
    (k*n + j)*n + i.
    """
    g = np.linspace(0.0, side, n)
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    coords = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    kk, jj, ii = np.meshgrid(np.arange(n - 1), np.arange(n - 1), np.arange(n - 1), indexing="ij")
    ii, jj, kk = ii.ravel(), jj.ravel(), kk.ravel()

    def nid(a, b, c):
        return ((kk + c) * n + (jj + b)) * n + (ii + a)

    corners = {(a, b, c): nid(a, b, c) for a in (0, 1) for b in (0, 1) for c in (0, 1)}
    parity = (ii + jj + kk) % 2
    tets = []
    for flip in (0, 1):
        # local corners whose global parity is even
        even = [abc for abc in corners if (sum(abc) + flip) % 2 == 0]
        odd = [abc for abc in corners if (sum(abc) + flip) % 2 == 1]
        sel = parity == flip
        cell_tets = [even]
        for o in odd:
            nb = [e for e in even if sum(abs(np.subtract(o, e))) == 1]
            cell_tets.append([o] + nb)
        tets.append((sel, cell_tets))
    out = np.zeros((ii.size, 5, 4), dtype=np.int32)
    for sel, cell_tets in tets:
        for t, verts in enumerate(cell_tets):
            for v, abc in enumerate(verts):
                out[sel, t, v] = corners[abc][sel]
    return coords, out.reshape(-1, 4)


def smoothed_gaussian(rng, shape, width):
    """N(0,1) field smoothed by a Gaussian of std `width` cells, renormalised to unit std."""
    g = gaussian_filter(rng.standard_normal(shape), sigma=width, mode="reflect")
    return (g - g.mean()) / g.std()


def fiber_angles_2d(rng, ncx, ncy, width):
    """Per-cell fibre angle: i.i.d. U[0, pi) angles, smoothed as the doubled-angle vector field."""
    psi = rng.uniform(0.0, np.pi, size=(ncy, ncx))
    c = gaussian_filter(np.cos(2 * psi), sigma=width, mode="reflect")
    s = gaussian_filter(np.sin(2 * psi), sigma=width, mode="reflect")
    return 0.5 * np.arctan2(s, c)


def rotated_tensor_2d(phi, d_long, d_trans):
    """D = R(phi) diag(d_long, d_trans) R(phi)^T, one 2x2 tensor per angle."""
    c, s = np.cos(phi), np.sin(phi)
    D = np.empty(phi.shape + (2, 2))
    D[..., 0, 0] = d_long * c * c + d_trans * s * s
    D[..., 1, 1] = d_long * s * s + d_trans * c * c
    D[..., 0, 1] = D[..., 1, 0] = (d_long - d_trans) * c * s
    return D


def fiber_tensor_3d(fdir, d_long, d_trans):
    """D = d_trans I + (d_long - d_trans) f f^T for unit fibre directions f [E, 3]."""
    D = d_trans * np.broadcast_to(np.eye(3), fdir.shape[:-1] + (3, 3)).copy()
    D += (d_long - d_trans) * fdir[..., :, None] * fdir[..., None, :]
    return D
