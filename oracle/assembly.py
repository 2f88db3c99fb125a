"""P1 finite-element assembly on simplices (oracle; test infrastructure).

Sec. 2.2 (eq. "abstract monodomain"): Lagrange P1 elements turn the
monodomain equation into M v' = -A v - b(v, w).  This module builds

* the row-sum lumped mass  ML_i = sum_{T containing i} |T| / (d + 1),
* the stiffness A = sum_T sigma_T Khat_T, where Khat_T = |T| G_T D_T G_T^T is
  the element stiffness for the element's unit conductivity tensor D_T,
  G_T holds the (constant) gradients of the barycentric coordinates, and
  sigma_T is the mean of the nodal conductivity multipliers over T's
  vertices (exact integration of a P1-interpolated scalar multiplier),
* dA/dsigma_n = sum_{T containing n} Khat_T / (d + 1), used by the
  tangent-linear model.

With beta * C_m = 1 the reaction term uses nodal quadrature, b = ML * I.
Elements are given as global vertex ids (several independent instances may
share one node numbering; they simply never share an element).
"""
import math

import numpy as np
import scipy.sparse as sp


def element_geometry(coords, elems):
    """Return (volumes [E], gradients [E, d+1, d]) of P1 barycentric functions."""
    coords = np.asarray(coords, dtype=np.float64)
    elems = np.asarray(elems, dtype=np.int64)
    d = coords.shape[1]
    X = coords[elems]                                # [E, d+1, d]
    Ed = X[:, 1:, :] - X[:, :1, :]                   # rows are edge vectors x_i - x_0
    det = np.linalg.det(Ed)
    vol = np.abs(det) / math.factorial(d)
    # lambda_i (i >= 1) = e_i . Ed^{-T} (x - x_0)  =>  grad lambda_i = row i of inv(Ed)^T
    inv = np.linalg.inv(Ed)                          # [E, d, d]
    g_rest = np.transpose(inv, (0, 2, 1))            # grad lambda_i for i = 1..d as rows
    g0 = -g_rest.sum(axis=1, keepdims=True)
    grads = np.concatenate([g0, g_rest], axis=1)     # [E, d+1, d]
    return vol, grads


def element_stiffness(coords, elems, elem_tensor):
    """Khat_T = |T| G_T D_T G_T^T for each element, shape [E, d+1, d+1]."""
    vol, G = element_geometry(coords, elems)
    D = np.asarray(elem_tensor, dtype=np.float64)
    return vol[:, None, None] * np.einsum("eia,eab,ejb->eij", G, D, G)


def lumped_mass(coords, elems, n_nodes):
    vol, _ = element_geometry(coords, elems)
    elems = np.asarray(elems, dtype=np.int64)
    d1 = elems.shape[1]
    return np.bincount(elems.ravel(), weights=np.repeat(vol / d1, d1), minlength=n_nodes)


def element_sigma(elems, node_sigma):
    return np.asarray(node_sigma, dtype=np.float64)[np.asarray(elems)].mean(axis=1)


def stiffness(coords, elems, elem_tensor, node_sigma, n_nodes):
    """Global stiffness A (scipy CSR, duplicates summed)."""
    elems = np.asarray(elems, dtype=np.int64)
    Khat = element_stiffness(coords, elems, elem_tensor)
    vals = element_sigma(elems, node_sigma)[:, None, None] * Khat
    d1 = elems.shape[1]
    rows = np.repeat(elems, d1, axis=1).ravel()
    cols = np.tile(elems, (1, d1)).ravel()
    A = sp.coo_matrix((vals.ravel(), (rows, cols)), shape=(n_nodes, n_nodes)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return A


def stiffness_sigma_derivative(coords, elems, elem_tensor, n_nodes, direction):
    """dA[direction] = sum_n direction_n dA/dsigma_n (a sparse matrix)."""
    elems = np.asarray(elems, dtype=np.int64)
    Khat = element_stiffness(coords, elems, elem_tensor)
    dsig = element_sigma(elems, direction)
    vals = dsig[:, None, None] * Khat
    d1 = elems.shape[1]
    rows = np.repeat(elems, d1, axis=1).ravel()
    cols = np.tile(elems, (1, d1)).ravel()
    return sp.coo_matrix((vals.ravel(), (rows, cols)), shape=(n_nodes, n_nodes)).tocsr()
