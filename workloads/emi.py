"""Cell-by-cell (EMI) workload: a rectangular array of myocytes in extracellular space.

Input arrays only (mesh, membrane and gap-junction node pairs, their lumped
measures, coefficients); no arithmetic of the method.

Geometry (lengths in cm): an nc x nr array of rectangular cells of size
cell_len x cell_h separated by gaps of width `gap`, with a margin of `gap`
around the array.  Each cell carries an nx x ny tensor grid of
intracellular nodes.  The extracellular nodes are the points of the global
tensor grid (all cell grid lines plus the outer boundary lines) that are not
strictly inside a cell; the cell boundary points therefore exist twice, once
as intracellular and once as extracellular node (a membrane site).  Every
grid rectangle is split along its (i,j)-(i+1,j+1) diagonal into two P1
triangles; extracellular triangles are those of grid rectangles outside the
cells.

Couplings:
- membrane sites: (intracellular node, extracellular node, lumped membrane
  length: half of each adjacent boundary segment of the cell);
- gap junctions: the nodes of a cell's right end face paired with those of
  the left end face of the next cell in its row (lumped face lengths);
- Robin boundary: lumped length of the outer boundary at each extracellular
  node on it (0 elsewhere).
"""
from dataclasses import dataclass, field

import numpy as np

from .configs import AP_PARAMS


@dataclass
class EmiProblem:
    name: str
    coords: np.ndarray          # [N, 2]
    elems: np.ndarray           # [E, 3] int32
    elem_tensor: np.ndarray     # [E, 2, 2] conductivity tensors (sigma I)
    node_sigma: np.ndarray      # [N] multipliers (ones)
    node_cell: np.ndarray       # [N] cell id, -1 extracellular
    mem_intra: np.ndarray       # [S] int32
    mem_extra: np.ndarray       # [S] int32
    mem_len: np.ndarray         # [S]
    gap_a: np.ndarray           # [G] int32
    gap_b: np.ndarray           # [G] int32
    gap_len: np.ndarray         # [G]
    robin_len: np.ndarray       # [N]
    cm: float                   # membrane capacitance
    g_gap: float                # gap-junction conductance per length
    eps: float                  # Robin coefficient
    ionic: np.ndarray           # [1, 6] Aliev-Panfilov parameters
    M: int
    K: int
    dt: float
    n_steps: int
    theta: float
    cg_rtol: float = 1e-12
    cg_maxit: int = 20000
    stimuli: list = field(default_factory=list)   # (t_on, int32 nodes, value)
    v_init: np.ndarray = None   # initial potentials u [N]
    w_init: np.ndarray = None   # initial gating [N] (meaningful at membrane sites)

    @property
    def N(self):
        return self.coords.shape[0]

    @property
    def n_inst(self):
        return 1

    @property
    def node_off(self):
        return np.array([0, self.N], dtype=np.int64)

    @property
    def elem_off(self):
        return np.array([0, self.elems.shape[0]], dtype=np.int64)


def _lumped(xs):
    """Half of each adjacent segment of the ascending points xs."""
    d = np.diff(xs)
    out = np.zeros(len(xs))
    out[:-1] += d / 2
    out[1:] += d / 2
    return out


def emi_mesh(nc, nr, nx, ny, cell_len, cell_h, gap):
    """Arrays of the cell array geometry (see the module docstring)."""
    xs = [0.0]
    for c in range(nc):
        x0 = gap + c * (cell_len + gap)
        xs += list(x0 + np.linspace(0.0, cell_len, nx))
    xs.append(nc * (cell_len + gap) + gap)
    ys = [0.0]
    for r in range(nr):
        y0 = gap + r * (cell_h + gap)
        ys += list(y0 + np.linspace(0.0, cell_h, ny))
    ys.append(nr * (cell_h + gap) + gap)
    xs, ys = np.array(xs), np.array(ys)
    NX, NY = len(xs), len(ys)

    def local(g, n, n_lines):
        """(cell index, local index) of global line g, (-1, -1) for the outer lines."""
        inner = (g >= 1) & (g <= n_lines - 2)
        return np.where(inner, (g - 1) // n, -1), np.where(inner, (g - 1) % n, -1)

    gx, gy = np.meshgrid(np.arange(NX), np.arange(NY), indexing="xy")   # [NY, NX]
    cx, ix = local(gx, nx, NX)
    cy, iy = local(gy, ny, NY)
    interior = (cx >= 0) & (cy >= 0) & (ix >= 1) & (ix <= nx - 2) & (iy >= 1) & (iy <= ny - 2)
    ext_id = -np.ones((NY, NX), dtype=np.int64)
    ext_id[~interior] = np.arange(int((~interior).sum()))
    n_ext = int((~interior).sum())
    coords = [np.stack([np.broadcast_to(xs, (NY, NX))[~interior], np.broadcast_to(ys[:, None], (NY, NX))[~interior]],
                       axis=1)]

    # extracellular triangles: grid rectangles not inside a cell
    ex_tris = []
    for j in range(NY - 1):
        for i in range(NX - 1):
            inside = (cx[j, i] >= 0 and cx[j, i] == cx[j, i + 1] and cy[j, i] >= 0 and cy[j, i] == cy[j + 1, i]
                      and ix[j, i] <= nx - 2 and iy[j, i] <= ny - 2)
            if inside:
                continue
            a, b, c_, d = ext_id[j, i], ext_id[j, i + 1], ext_id[j + 1, i + 1], ext_id[j + 1, i]
            ex_tris.append((a, b, c_))
            ex_tris.append((a, c_, d))
    ex_tris = np.array(ex_tris, dtype=np.int64)

    # intracellular nodes and triangles, cell by cell
    n_cell_nodes = nx * ny
    in_tris, node_cell = [], [-np.ones(n_ext, dtype=np.int64)]
    mem_i, mem_e, mem_l = [], [], []
    lx = _lumped(np.linspace(0.0, cell_len, nx))
    ly = _lumped(np.linspace(0.0, cell_h, ny))
    base = n_ext
    for r in range(nr):
        for c in range(nc):
            cell = r * nc + c
            gx0, gy0 = 1 + c * nx, 1 + r * ny
            coords.append(np.stack([np.tile(xs[gx0:gx0 + nx], ny), np.repeat(ys[gy0:gy0 + ny], nx)], axis=1))
            node_cell.append(np.full(n_cell_nodes, cell))
            lid = base + np.arange(n_cell_nodes).reshape(ny, nx)
            for j in range(ny - 1):
                for i in range(nx - 1):
                    a, b, c_, d = lid[j, i], lid[j, i + 1], lid[j + 1, i + 1], lid[j + 1, i]
                    in_tris.append((a, b, c_))
                    in_tris.append((a, c_, d))
            for j in range(ny):
                for i in range(nx):
                    on_x, on_y = i in (0, nx - 1), j in (0, ny - 1)
                    if not (on_x or on_y):
                        continue
                    length = (lx[i] if on_y else 0.0) + (ly[j] if on_x else 0.0)
                    mem_i.append(lid[j, i])
                    mem_e.append(ext_id[gy0 + j, gx0 + i])
                    mem_l.append(length)
            base += n_cell_nodes
    coords = np.concatenate(coords)
    N = coords.shape[0]

    # gap junctions between neighbouring cells of a row (end faces)
    gap_a, gap_b, gap_l = [], [], []
    for r in range(nr):
        for c in range(nc - 1):
            left = n_ext + (r * nc + c) * n_cell_nodes
            right = n_ext + (r * nc + c + 1) * n_cell_nodes
            for j in range(ny):
                gap_a.append(left + j * nx + (nx - 1))
                gap_b.append(right + j * nx)
                gap_l.append(ly[j])

    # Robin boundary: lumped length along the outer boundary
    robin = np.zeros(N)
    bx, by = _lumped(xs), _lumped(ys)
    for i in range(NX):
        robin[ext_id[0, i]] += bx[i]
        robin[ext_id[NY - 1, i]] += bx[i]
    for j in range(NY):
        robin[ext_id[j, 0]] += by[j]
        robin[ext_id[j, NX - 1]] += by[j]

    elems = np.concatenate([ex_tris, np.array(in_tris, dtype=np.int64)]).astype(np.int32)
    elem_cell = np.concatenate([-np.ones(len(ex_tris), dtype=np.int64),
                                np.concatenate(node_cell)[np.array(in_tris)[:, 0]]])
    return dict(coords=coords, elems=elems, elem_cell=elem_cell, node_cell=np.concatenate(node_cell),
                mem_intra=np.array(mem_i, dtype=np.int32), mem_extra=np.array(mem_e, dtype=np.int32),
                mem_len=np.array(mem_l), gap_a=np.array(gap_a, dtype=np.int32),
                gap_b=np.array(gap_b, dtype=np.int32), gap_len=np.array(gap_l), robin_len=robin,
                width=xs[-1], height=ys[-1])


def config3(nc=64, nr=16, nx=33, ny=9, seed=3, theta=1e-6, n_steps=1000, M=3, K=4, dt=0.05,
            cell_len=100e-4, cell_h=16e-4, gap=2e-4, sigma_i=3.0, sigma_e=20.0, cm=1.0, g_gap=0.5,
            eps=1e-3, spread=1.2):
    """The cell-by-cell workload (lengths in cm, conductivities in mS/cm,
    capacitance in uF/cm^2, time in ms): intracellular conductivity
    sigma_i * spread^xi per cell (xi ~ N(0,1), seed), extracellular sigma_e,
    stimulus u = 1 on the intracellular nodes of the first cell column at t = 0."""
    g = emi_mesh(nc, nr, nx, ny, cell_len, cell_h, gap)
    rng = np.random.default_rng(seed)
    cell_sigma = sigma_i * np.exp(np.log(spread) * rng.standard_normal(nc * nr))
    sig = np.where(g["elem_cell"] >= 0, cell_sigma[np.maximum(g["elem_cell"], 0)], sigma_e)
    tensor = sig[:, None, None] * np.eye(2)[None]
    N = g["coords"].shape[0]
    first_col = np.nonzero((g["node_cell"] >= 0) & (g["node_cell"] % nc == 0))[0].astype(np.int32)
    return EmiProblem(name="2d-emi", coords=g["coords"], elems=g["elems"], elem_tensor=tensor,
                      node_sigma=np.ones(N), node_cell=g["node_cell"], mem_intra=g["mem_intra"],
                      mem_extra=g["mem_extra"], mem_len=g["mem_len"], gap_a=g["gap_a"], gap_b=g["gap_b"],
                      gap_len=g["gap_len"], robin_len=g["robin_len"], cm=cm, g_gap=g_gap, eps=eps,
                      ionic=np.array([AP_PARAMS]), M=M, K=K, dt=dt, n_steps=n_steps, theta=theta,
                      stimuli=[(0.0, first_col, 1.0)], v_init=np.zeros(N), w_init=np.zeros(N))


# ------------------------------------------------------------------ 3D

# The Kuhn split of a grid hexahedron: for every ordering (a, b, c) of the
# axes the tetrahedron 000, e_a, e_a + e_b, 111 (corners as (dx, dy, dz)).
# Every face of the hexahedron is then split along its diagonal from the
# low to the high corner, so neighbouring hexahedra match.
_KUHN = []
for _a, _b, _c in ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)):
    _p1 = [0, 0, 0]
    _p1[_a] = 1
    _p2 = list(_p1)
    _p2[_b] = 1
    _KUHN.append(((0, 0, 0), tuple(_p1), tuple(_p2), (1, 1, 1)))


def _face_lumped(us, vs):
    """P1-lumped area per node of a rectangular face gridded by the ascending
    points us x vs, each grid rectangle split into two triangles along its
    low-to-high diagonal: a third of each adjacent triangle's area.
    Returns [len(vs), len(us)]."""
    out = np.zeros((len(vs), len(us)))
    du, dv = np.diff(us), np.diff(vs)
    half = 0.5 * dv[:, None] * du[None, :] / 3.0   # a third of each triangle
    # triangle (00, 10, 11) and (00, 01, 11): corners 00 and 11 in both
    out[:-1, :-1] += 2 * half
    out[1:, 1:] += 2 * half
    out[:-1, 1:] += half
    out[1:, :-1] += half
    return out


def emi_mesh3d(nc, nr, nl, nx, ny, nz, cell_len, cell_h, cell_d, gap):
    """Arrays of a 3D cell array: nc x nr x nl brick cells of size cell_len x
    cell_h x cell_d with nx x ny x nz intracellular nodes each, gaps of width
    `gap` between cells and around the array (one element wide), the same
    node and coupling conventions as the 2D mesh with areas for lengths, and
    every grid hexahedron split into six tetrahedra (Kuhn split)."""
    def lines(n_cells, n, size):
        xs = [0.0]
        for c in range(n_cells):
            x0 = gap + c * (size + gap)
            xs += list(x0 + np.linspace(0.0, size, n))
        xs.append(n_cells * (size + gap) + gap)
        return np.array(xs)

    xs, ys, zs = lines(nc, nx, cell_len), lines(nr, ny, cell_h), lines(nl, nz, cell_d)
    NX, NY, NZ = len(xs), len(ys), len(zs)

    def local(g, n, n_lines):
        inner = (g >= 1) & (g <= n_lines - 2)
        return np.where(inner, (g - 1) // n, -1), np.where(inner, (g - 1) % n, -1)

    gz, gy, gx = np.meshgrid(np.arange(NZ), np.arange(NY), np.arange(NX), indexing="ij")   # [NZ, NY, NX]
    cx, ix = local(gx, nx, NX)
    cy, iy = local(gy, ny, NY)
    cz, iz = local(gz, nz, NZ)
    interior = ((cx >= 0) & (cy >= 0) & (cz >= 0) & (ix >= 1) & (ix <= nx - 2) & (iy >= 1) & (iy <= ny - 2)
                & (iz >= 1) & (iz <= nz - 2))
    ext_id = -np.ones((NZ, NY, NX), dtype=np.int64)
    n_ext = int((~interior).sum())
    ext_id[~interior] = np.arange(n_ext)
    coords = [np.stack([np.broadcast_to(xs, (NZ, NY, NX))[~interior],
                        np.broadcast_to(ys[None, :, None], (NZ, NY, NX))[~interior],
                        np.broadcast_to(zs[:, None, None], (NZ, NY, NX))[~interior]], axis=1)]

    def hex_inside(lo_line, c_arr, i_arr, n):
        """Per hexahedron layer [lo, lo + 1] of one axis: the cell index when both lines belong to one cell, else -1."""
        same = (c_arr[:-1] >= 0) & (c_arr[:-1] == c_arr[1:]) & (i_arr[:-1] <= n - 2)
        return np.where(same, c_arr[:-1], -1)

    hx = hex_inside(None, cx[0, 0, :], ix[0, 0, :], nx)
    hy = hex_inside(None, cy[0, :, 0], iy[0, :, 0], ny)
    hz = hex_inside(None, cz[:, 0, 0], iz[:, 0, 0], nz)

    def tets_of(ids):
        """Six tetrahedra of every hexahedron of the node id grid ids [Z, Y, X]."""
        out = []
        for corners in _KUHN:
            out.append(np.stack([ids[dz:ids.shape[0] - 1 + dz, dy:ids.shape[1] - 1 + dy, dx:ids.shape[2] - 1 + dx]
                                 for dx, dy, dz in corners], axis=-1))
        return out

    # extracellular tetrahedra: hexahedra not inside a cell
    inside = (hz[:, None, None] >= 0) & (hy[None, :, None] >= 0) & (hx[None, None, :] >= 0)
    ex_tets = np.concatenate([t[~inside] for t in tets_of(ext_id)])

    n_cell_nodes = nx * ny * nz
    in_tets, node_cell, elem_cell = [], [-np.ones(n_ext, dtype=np.int64)], []
    mem_i, mem_e, mem_l = [], [], []
    px, py, pz = np.linspace(0.0, cell_len, nx), np.linspace(0.0, cell_h, ny), np.linspace(0.0, cell_d, nz)
    f_yz = _face_lumped(py, pz)   # end faces x = const: [nz, ny]
    f_xz = _face_lumped(px, pz)   # faces y = const: [nz, nx]
    f_xy = _face_lumped(px, py)   # faces z = const: [ny, nx]
    area = np.zeros((nz, ny, nx))
    area[:, :, 0] += f_yz
    area[:, :, -1] += f_yz
    area[:, 0, :] += f_xz
    area[:, -1, :] += f_xz
    area[0, :, :] += f_xy
    area[-1, :, :] += f_xy
    on_surface = np.zeros((nz, ny, nx), dtype=bool)
    on_surface[[0, -1], :, :] = True
    on_surface[:, [0, -1], :] = True
    on_surface[:, :, [0, -1]] = True
    base = n_ext
    for l in range(nl):
        for r in range(nr):
            for c in range(nc):
                cell = (l * nr + r) * nc + c
                gx0, gy0, gz0 = 1 + c * nx, 1 + r * ny, 1 + l * nz
                zz, yy, xx = np.meshgrid(zs[gz0:gz0 + nz], ys[gy0:gy0 + ny], xs[gx0:gx0 + nx], indexing="ij")
                coords.append(np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1))
                node_cell.append(np.full(n_cell_nodes, cell))
                lid = base + np.arange(n_cell_nodes).reshape(nz, ny, nx)
                t = np.concatenate([q.reshape(-1, 4) for q in tets_of(lid)])
                in_tets.append(t)
                elem_cell.append(np.full(len(t), cell))
                ext = ext_id[gz0:gz0 + nz, gy0:gy0 + ny, gx0:gx0 + nx]
                mem_i.append(lid[on_surface])
                mem_e.append(ext[on_surface])
                mem_l.append(area[on_surface])
                base += n_cell_nodes
    coords = np.concatenate(coords)
    N = coords.shape[0]

    # gap junctions between neighbouring cells of a row (end faces x = const)
    gap_a, gap_b, gap_l = [], [], []
    for l in range(nl):
        for r in range(nr):
            for c in range(nc - 1):
                left = n_ext + ((l * nr + r) * nc + c) * n_cell_nodes
                right = left + n_cell_nodes
                k, j = np.meshgrid(np.arange(nz), np.arange(ny), indexing="ij")
                gap_a.append((left + (k * ny + j) * nx + (nx - 1)).ravel())
                gap_b.append((right + (k * ny + j) * nx).ravel())
                gap_l.append(f_yz.ravel())

    # Robin boundary: lumped area of the outer boundary faces
    robin = np.zeros(N)
    for ids, face in ((ext_id[:, :, 0], _face_lumped(ys, zs)), (ext_id[:, :, -1], _face_lumped(ys, zs)),
                      (ext_id[:, 0, :], _face_lumped(xs, zs)), (ext_id[:, -1, :], _face_lumped(xs, zs)),
                      (ext_id[0, :, :], _face_lumped(xs, ys)), (ext_id[-1, :, :], _face_lumped(xs, ys))):
        np.add.at(robin, ids.ravel(), face.ravel())

    elems = np.concatenate([ex_tets] + in_tets).astype(np.int64)
    # orient every tetrahedron positively
    x = coords[elems]
    det = np.einsum("ij,ij->i", np.cross(x[:, 1] - x[:, 0], x[:, 2] - x[:, 0]), x[:, 3] - x[:, 0])
    flip = det < 0
    elems[flip, 1], elems[flip, 2] = elems[flip, 2].copy(), elems[flip, 1].copy()
    return dict(coords=coords, elems=elems.astype(np.int32),
                elem_cell=np.concatenate([-np.ones(len(ex_tets), dtype=np.int64)] + elem_cell),
                node_cell=np.concatenate(node_cell),
                mem_intra=np.concatenate(mem_i).astype(np.int32), mem_extra=np.concatenate(mem_e).astype(np.int32),
                mem_len=np.concatenate(mem_l), gap_a=np.concatenate(gap_a).astype(np.int32) if gap_a else
                np.zeros(0, np.int32), gap_b=np.concatenate(gap_b).astype(np.int32) if gap_b else np.zeros(0, np.int32),
                gap_len=np.concatenate(gap_l) if gap_l else np.zeros(0), robin_len=robin,
                size=(xs[-1], ys[-1], zs[-1]))


def config5(nc=8, nr=3, nl=2, nx=33, ny=9, nz=9, seed=5, theta=1e-6, n_steps=1000, M=3, K=4, dt=0.05,
            cell_len=100e-4, cell_h=16e-4, cell_d=16e-4, gap=2e-4, sigma_i=3.0, sigma_e=20.0, cm=1.0,
            g_gap=0.5, eps=1e-3, spread=1.2):
    """The 3D cell-by-cell workload: an 8 x 3 x 2 array of 100 x 16 x 16 um
    myocytes (33 x 9 x 9 nodes each) in extracellular space, P1 tetrahedra;
    coefficients and stimulus as in the 2D workload (the first cell column)."""
    g = emi_mesh3d(nc, nr, nl, nx, ny, nz, cell_len, cell_h, cell_d, gap)
    rng = np.random.default_rng(seed)
    cell_sigma = sigma_i * np.exp(np.log(spread) * rng.standard_normal(nc * nr * nl))
    sig = np.where(g["elem_cell"] >= 0, cell_sigma[np.maximum(g["elem_cell"], 0)], sigma_e)
    tensor = sig[:, None, None] * np.eye(3)[None]
    N = g["coords"].shape[0]
    first_col = np.nonzero((g["node_cell"] >= 0) & (g["node_cell"] % nc == 0))[0].astype(np.int32)
    return EmiProblem(name="3d-emi", coords=g["coords"], elems=g["elems"], elem_tensor=tensor,
                      node_sigma=np.ones(N), node_cell=g["node_cell"], mem_intra=g["mem_intra"],
                      mem_extra=g["mem_extra"], mem_len=g["mem_len"], gap_a=g["gap_a"], gap_b=g["gap_b"],
                      gap_len=g["gap_len"], robin_len=g["robin_len"], cm=cm, g_gap=g_gap, eps=eps,
                      ionic=np.array([AP_PARAMS]), M=M, K=K, dt=dt, n_steps=n_steps, theta=theta,
                      stimuli=[(0.0, first_col, 1.0)], v_init=np.zeros(N), w_init=np.zeros(N))
