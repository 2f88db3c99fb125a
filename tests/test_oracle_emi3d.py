"""Pins of the cell-by-cell (EMI) oracle on the 3D cell array (P1 tetrahedra).

The same facts as in 2D, with areas for lengths:
- the mesh fills the box exactly with positively oriented tetrahedra, and
  the lumped membrane, gap-face and outer-boundary measures (computed by the
  oracle from the mesh's boundary triangles) sum to the exact areas, take
  their closed forms at face-interior sites (hu hv: six triangles of area
  hu hv / 2, a third each) and at the cells' two diagonal corners, and agree
  with the workload's arrays;
- the membrane jump mass annihilates constants and gives each cell's
  indicator the energy C_m x (cell surface area);
- A maps constants to the Robin term only (eps x box surface in total),
  annihilates affine functions on interior rows of every subdomain, and a
  cell's indicator only feels the gap junctions of its end faces;
- converged sweeps reproduce the Radau-IIA collocation solution (Newton);
- in the lumped limit one cell obeys the membrane ODE (SciPy's Radau).
"""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import ionic
from oracle.emi import EMI, build, collocation_solution, run
from workloads.emi import config5

L, H, D, GAP = 100e-4, 16e-4, 16e-4, 2e-4


def small(**kw):
    base = dict(nc=2, nr=2, nl=1, nx=4, ny=3, nz=3)
    base.update(kw)
    return config5(**base)


def box(nc, nr, nl):
    return nc * (L + GAP) + GAP, nr * (H + GAP) + GAP, nl * (D + GAP) + GAP


def test_mesh_measures():
    P = small()
    mod = EMI(P)
    W, Hb, Db = box(2, 2, 1)
    x = P.coords[P.elems]
    det = np.einsum("ij,ij->i", np.cross(x[:, 1] - x[:, 0], x[:, 2] - x[:, 0]), x[:, 3] - x[:, 0])
    assert det.min() > 0
    assert abs(det.sum() / 6 - W * Hb * Db) <= 1e-12 * W * Hb * Db
    assert abs(mod.robin_len.sum() - 2 * (W * Hb + W * Db + Hb * Db)) <= 1e-14
    assert abs(mod.mem_len.sum() - 4 * 2 * (L * H + L * D + H * D)) <= 1e-14
    assert abs(mod.gap_len.sum() - 2 * H * D) <= 1e-15   # one neighbour pair per row, two rows
    for a, b in ((mod.mem_len, P.mem_len), (mod.gap_len, P.gap_len), (mod.robin_len, P.robin_len)):
        assert np.allclose(a, b, rtol=1e-13, atol=0)


def test_lumped_measures_per_site():
    nx, ny, nz = 5, 4, 4
    P = small(nx=nx, ny=ny, nz=nz)
    mod = EMI(P)
    hx, hy, hz = L / (nx - 1), H / (ny - 1), D / (nz - 1)
    xyz = P.coords[P.mem_intra]
    cell = P.node_cell[P.mem_intra]
    for c in np.unique(cell):
        s = cell == c
        lo, hi = xyz[s].min(axis=0), xyz[s].max(axis=0)
        at_lo = np.isclose(xyz[s], lo, rtol=0, atol=1e-12)
        at_hi = np.isclose(xyz[s], hi, rtol=0, atol=1e-12)
        faces = (at_lo | at_hi).sum(axis=1)
        # on one face only: hu hv of that face's grid
        one = faces == 1
        ax = np.argmax((at_lo | at_hi)[one], axis=1)
        area = np.array([hy * hz, hx * hz, hx * hy])[ax]
        assert one.sum() > 10 and np.allclose(mod.mem_len[s][one], area, rtol=1e-13, atol=0)
        # the low and the high corner: the diagonal end of all three faces'
        # grid squares, two triangles each: (hx hy + hx hz + hy hz) / 3
        corner = np.all(at_lo, axis=1) | np.all(at_hi, axis=1)
        assert corner.sum() == 2
        assert np.allclose(mod.mem_len[s][corner], (hx * hy + hx * hz + hy * hz) / 3, rtol=1e-13, atol=0)
    # gap faces (x = const): interior nodes hy hz, total H D per pair of faces
    gyz = P.coords[P.gap_a, 1:]
    inner = np.zeros(len(P.gap_a), dtype=bool)
    for c in np.unique(P.node_cell[P.gap_a]):
        s = P.node_cell[P.gap_a] == c
        lo, hi = gyz[s].min(axis=0), gyz[s].max(axis=0)
        inner[np.nonzero(s)[0]] = np.all((gyz[s] > lo + 1e-12) & (gyz[s] < hi - 1e-12), axis=1)
    assert inner.sum() > 0 and np.allclose(mod.gap_len[inner], hy * hz, rtol=1e-13, atol=0)


def test_membrane_mass():
    P = small()
    Mm = EMI(P).M.toarray()
    assert np.allclose(Mm, Mm.T, atol=0)
    assert np.abs(Mm @ np.ones(P.N)).max() <= 1e-15 * np.abs(Mm).max()
    assert np.linalg.eigvalsh(Mm).min() > -1e-15 * P.N * np.abs(Mm).max()
    surf = 2 * (L * H + L * D + H * D)
    for c in range(4):
        ind = (P.node_cell == c).astype(float)
        assert abs(ind @ Mm @ ind - P.cm * surf) <= 1e-12 * surf


def test_stiffness_constants_and_affine_functions():
    P = small()
    A = EMI(P).A
    # the plain element products sigma (G_a . G_b) are symmetric to rounding
    assert abs(A - A.T).max() <= 4e-16 * abs(A).max()
    assert np.allclose(A @ np.ones(P.N), P.eps * EMI(P).robin_len, rtol=0, atol=1e-15 * 24 * abs(A).max())
    W, Hb, Db = box(2, 2, 1)
    assert abs(np.ones(P.N) @ A @ np.ones(P.N) - P.eps * 2 * (W * Hb + W * Db + Hb * Db)) \
        <= 1e-15 * A.nnz * abs(A).max()
    Pa = small(nx=6, ny=5, nz=4)   # enough interior nodes for the affine check
    Aa = EMI(Pa).A
    x, y, z = Pa.coords.T
    u = 2 * x - 3 * y + z
    interior = np.ones(Pa.N, dtype=bool)
    for a in (Pa.mem_intra, Pa.mem_extra, Pa.gap_a, Pa.gap_b):
        interior[a] = False
    interior[Pa.robin_len > 0] = False
    assert interior.sum() > 20
    assert np.abs((Aa @ u)[interior]).max() <= 1e-12 * np.abs(Aa).max() * np.abs(u).max()
    for c in range(4):
        ind = (P.node_cell == c).astype(float)
        n_nb = 1   # two cells per row: every cell has one neighbour
        assert abs(ind @ (A @ ind) - P.g_gap * H * D * n_nb) <= 1e-12 * abs(A).max() * A.nnz * 1e-3


@pytest.mark.parametrize("M", [2, 3])
def test_converged_sweeps_equal_collocation_solution(M):
    P = config5(nc=2, nr=1, nl=1, nx=3, ny=3, nz=3, M=M, dt=0.05, theta=0.0)
    u0 = np.zeros(P.N)
    u0[P.stimuli[0][1]] = 1.0
    w0 = np.full(len(P.mem_intra), 0.05)
    sdc = build(P, direct=True)
    st = sdc.spread(u0, w0)
    idx = np.arange(P.N)
    for _ in range(60):
        sdc.sweep(st, idx)
    Uc, Wc = collocation_solution(sdc.model, M, P.dt, u0, w0)
    d = st["u"] - Uc
    si, se = sdc.model.si, sdc.model.se
    # the constant of the potentials is fixed only by the weak Robin term
    assert np.abs(d[:, si] - d[:, se]).max() <= 1e-12
    assert np.abs(d - d.mean(axis=1, keepdims=True)).max() <= 1e-12 * np.abs(Uc).max()
    assert np.abs(d).max() <= 1e-8 * np.abs(Uc).max()
    assert np.abs(st["w"] - Wc).max() <= 1e-12 * max(np.abs(Wc).max(), 1.0)


def test_single_cell_lumped_limit_follows_membrane_ode():
    big = 1e6
    P = config5(nc=1, nr=1, nl=1, nx=4, ny=3, nz=3, sigma_i=big, sigma_e=big, eps=big, M=3, dt=0.02, theta=0.0)
    sdc = build(P, direct=True)
    u = np.zeros(P.N)
    u[P.node_cell == 0] = 0.3
    w = np.zeros(len(P.mem_intra))
    n_steps, K = 25, 12
    u, w, _ = run(sdc, u, w, n_steps, K)
    p = np.asarray(P.ionic[0])

    def rhs(t, y):
        v, g = y
        return [-ionic.current(v, g, p) / P.cm, ionic.rate(v, g, p)]

    ref = solve_ivp(rhs, (0.0, n_steps * P.dt), [0.3, 0.0], method="Radau", rtol=1e-12, atol=1e-14)
    v_end = u[P.mem_intra] - u[P.mem_extra]
    assert np.abs(v_end - ref.y[0, -1]).max() <= 1e-5
    assert np.abs(w - ref.y[1, -1]).max() <= 1e-5
    assert abs(v_end.mean() - 0.3) > 0.05


def test_tetrahedra_are_conforming():
    """Every triangle face of the tetrahedra is shared by two of them, except
    the faces on the box boundary and on cell surfaces (where intra- and
    extracellular nodes differ): a face seen once anywhere else would mean
    that neighbouring hexahedra cut a grid face along different diagonals."""
    nc, nr, nl = 2, 2, 1
    P = config5(nc=nc, nr=nr, nl=nl, nx=5, ny=4, nz=4)
    faces = {}
    for t in P.elems:
        for drop in range(4):
            f = tuple(sorted(np.delete(t, drop)))
            faces[f] = faces.get(f, 0) + 1
    assert max(faces.values()) == 2
    W, Hb, Db = box(nc, nr, nl)
    planes = [{0.0, W}, {0.0, Hb}, {0.0, Db}]
    for k, (n, size) in enumerate(((nc, L), (nr, H), (nl, D))):
        for c in range(n):
            planes[k] |= {GAP + c * (size + GAP), GAP + c * (size + GAP) + size}
    n_single = 0
    for f, n in faces.items():
        if n == 2:
            continue
        n_single += 1
        c = P.coords[list(f)]
        flat = [k for k in range(3) if np.ptp(c[:, k]) < 1e-12]
        assert len(flat) == 1
        k = flat[0]
        assert min(abs(c[0, k] - v) for v in planes[k]) < 1e-12
    # two triangles per boundary grid rectangle; cell surfaces seen from both sides
    nx, ny, nz = 5, 4, 4
    NX, NY, NZ = nc * nx + 2, nr * ny + 2, nl * nz + 2
    box_tris = 2 * 2 * ((NX - 1) * (NY - 1) + (NX - 1) * (NZ - 1) + (NY - 1) * (NZ - 1))
    cell_tris = 2 * 2 * 2 * ((nx - 1) * (ny - 1) + (nx - 1) * (nz - 1) + (ny - 1) * (nz - 1)) * nc * nr * nl
    assert n_single == box_tris + cell_tris
