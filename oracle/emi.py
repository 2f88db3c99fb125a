"""Adaptive IMEX SDC step for the cell-by-cell (EMI) system (oracle; test infrastructure).

Problem (Sec. 2.1, eq. cell-by-cell, weak form, and the discrete system of
eqs. abstract reaction diffusion / abstract gating): with P1 elements on
each subdomain (potentials discontinuous across membranes),

    M u' = -A u - b(u, w),          w_s' = R(v_s, w_s)  on membrane sites s,

where, for a membrane site s with intracellular node i(s), extracellular
node e(s) at the same position and lumped membrane length l_s,

    v_s  = u_i(s) - u_e(s)                                (transmembrane voltage)
    M    = C_m  sum_s l_s (e_i - e_e)(e_i - e_e)^T          (membrane "jump" mass)
    b    = sum_s l_s I(v_s, w_s) (e_i - e_e)                (ionic current)
    A    = sum_T sigma_T Khat_T  +  eps diag(robin_len)  +  g_gap sum_g l_g (e_a - e_b)(e_a - e_b)^T,

the last two terms being the Robin condition on the outer boundary and the
linear gap junctions between neighbouring cells (linear, so implicit with
the diffusion).  M is singular (only membrane nodes carry it): the system
is an index-1 DAE, and H_m = M + dt QI[m,m] A is SPD.

The sweep is the IMEX SDC of :mod:`oracle.sdc` with ML replaced by M and
ML*I by b (Sec. 3, eq. final-sdc, written for u):

    Phi_m = M (u0 - u_m) + dt sum_j Q[m,j] (-A u_j - b_j)
    Gam_m = w0 - w_m + dt sum_j Q[m,j] R_j                          (sites)
    dw_m  = Gam_m + dt sum_{j<m} QE[m,j] dR_j
    H_m du_m = Phi_m - dt sum_{j<m} QE[m,j] B(dI_j) - A (dt sum_{j<m} QI[m,j] du_j)

with B(dI) = sum_s l_s dI_s (e_i - e_e).  Adaptivity as for the monodomain
model, on the rows (nodes) of u.  Readings specific to this model: a
membrane site (its w, I, R) is updated in a sweep iff its intracellular
node is active; the changes dI, dR of the other sites count as zero; the
rule measures max_m |du_m| per node.
"""
import numpy as np
import scipy.sparse as sp
from scipy.sparse.linalg import splu

from . import ionic
from .assembly import stiffness
from .collocation import Collocation
from .pcg import jacobi_pcg
from .sdc import apply_stimuli


def _facets(elems):
    """Every facet of every simplex (a simplex without one vertex), vertex
    ids ascending, with the simplex it belongs to."""
    e = np.asarray(elems, dtype=np.int64)
    nv = e.shape[1]
    f = np.concatenate([np.delete(e, q, axis=1) for q in range(nv)])
    return np.sort(f, axis=1), np.tile(np.arange(e.shape[0]), nv)


def _facet_measure(coords, f):
    """Length of each edge (2D) or area of each triangle (3D)."""
    x = coords[f]
    if f.shape[1] == 2:
        return np.linalg.norm(x[:, 1] - x[:, 0], axis=1)
    return 0.5 * np.linalg.norm(np.cross(x[:, 1] - x[:, 0], x[:, 2] - x[:, 0]), axis=1)


def lumped_measures(coords, elems, node_cell, mem_intra, gap_a):
    """The P1-lumped measures of the cell-by-cell couplings, from the mesh.

    A coupling on a curve (2D) or surface (3D) is lumped like the mass: each
    boundary facet gives 1/d of its measure to each of its d vertices (the
    integral of the vertex's hat function over the facet).  The facets are
    found from the simplices: a cell's membrane is the set of facets that
    belong to exactly one of the cell's simplices; the outer boundary is the
    set of facets of exactly one extracellular simplex that lie in a face of
    the domain's bounding box; a gap-junction face of a cell is its membrane
    in the plane x = const through the node.  Returns (membrane measure of
    each site, at its intracellular node; gap-face measure of each pair, at
    its first node; outer-boundary measure of every node)."""
    coords = np.asarray(coords, dtype=np.float64)
    N, d = coords.shape
    f, owner = _facets(elems)
    cell = np.asarray(node_cell)[np.asarray(elems, dtype=np.int64)[:, 0]][owner]   # subdomain of each facet's simplex
    key = np.concatenate([cell[:, None], f], axis=1)
    _, inv, cnt = np.unique(key, axis=0, return_inverse=True, return_counts=True)
    boundary = cnt[inv.ravel()] == 1
    share = np.repeat(_facet_measure(coords, f) / d, d)
    x = coords[f]                                                # [F, d, d]

    def lump(mask):
        out = np.zeros(N)
        np.add.at(out, f[mask].ravel(), share.reshape(-1, d)[mask].ravel())
        return out

    membrane = boundary & (cell >= 0)
    lo, hi = coords.min(axis=0), coords.max(axis=0)
    on_box = np.zeros(len(f), dtype=bool)
    for ax in range(d):
        on_box |= np.all(x[:, :, ax] == lo[ax], axis=1) | np.all(x[:, :, ax] == hi[ax], axis=1)
    in_x_plane = np.all(x[:, :, 0] == x[:, :1, 0], axis=1)
    mem = lump(membrane)[np.asarray(mem_intra, dtype=np.int64)]
    gap = lump(membrane & in_x_plane)[np.asarray(gap_a, dtype=np.int64)]
    robin = lump(boundary & (cell < 0) & on_box)
    return mem, gap, robin


class EMI:
    """A, M, membrane sites and ionic parameters of a cell-by-cell mesh.

    The lumped membrane, gap-face and outer-boundary measures are computed
    here from the mesh (lumped_measures); the problem supplies only which
    node pairs are coupled."""

    def __init__(self, P):
        N = P.N
        self.N = N
        mem_len, gap_len, robin_len = lumped_measures(P.coords, P.elems, P.node_cell, P.mem_intra, P.gap_a)
        self.mem_len, self.gap_len, self.robin_len = mem_len, gap_len, robin_len
        A = stiffness(P.coords, P.elems, P.elem_tensor, P.node_sigma, N)
        ga, gb, gw = np.asarray(P.gap_a), np.asarray(P.gap_b), P.g_gap * gap_len
        rows = np.concatenate([ga, gb, ga, gb])
        cols = np.concatenate([ga, gb, gb, ga])
        vals = np.concatenate([gw, gw, -gw, -gw])
        Agap = sp.coo_matrix((vals, (rows, cols)), shape=(N, N))
        self.A = (A + Agap + sp.diags(P.eps * robin_len)).tocsr()
        si, se = np.asarray(P.mem_intra, dtype=np.int64), np.asarray(P.mem_extra, dtype=np.int64)
        ml = P.cm * mem_len
        rows = np.concatenate([si, se, si, se])
        cols = np.concatenate([si, se, se, si])
        vals = np.concatenate([ml, ml, -ml, -ml])
        self.M = sp.coo_matrix((vals, (rows, cols)), shape=(N, N)).tocsr()
        self.si, self.se = si, se
        self.l = mem_len
        self.S = si.size
        self.p = np.asarray(P.ionic[0], dtype=np.float64)[:, None]   # [6, 1] broadcast over sites

    def voltage(self, u, sites):
        return u[self.si[sites]] - u[self.se[sites]]

    def reaction(self, u, w_sites, sites):
        """(I, R) at the given sites from the potentials u and the sites' gating values."""
        v = self.voltage(u, sites)
        return ionic.current(v, w_sites, self.p), ionic.rate(v, w_sites, self.p)

    def bvec(self, I_sites):
        """sum_s l_s I_s (e_i - e_e): the nodal vector of a site quantity."""
        out = np.zeros(self.N)
        np.add.at(out, self.si, self.l * I_sites)
        np.add.at(out, self.se, -self.l * I_sites)
        return out


class EmiSDC:
    """IMEX SDC on Radau-IIA nodes for the EMI system, nested active node sets.

    ``direct=True`` solves the restricted systems with a sparse LU instead of
    Jacobi-PCG (same solution to rounding; for extreme test parameters).

    Optional energy-norm termination (Sec. 3.2, stated for the abstract form
    of both models): with tol_sdc > 0 the step ends after the first sweep k
    (k + 1 >= K_min) with  sum_m du_m^T H_m du_m <= ((1 - rho) / rho * tol_sdc)^2.
    """

    def __init__(self, model, M, dt, theta, cg_rtol=1e-12, cg_maxit=20000, direct=False, tol_sdc=0.0,
                 rho=0.05, K_min=1):
        self.model = model
        self.col = Collocation(M)
        self.M = M
        self.dt = float(dt)
        self.theta = float(theta)
        self.cg_rtol = cg_rtol
        self.cg_maxit = cg_maxit
        self.direct = direct
        self.tol_sdc = float(tol_sdc)
        self.rho = float(rho)
        self.K_min = int(K_min)
        self.H = [(model.M + self.dt * self.col.QI[m, m] * model.A).tocsr() for m in range(M)]

    def energy(self, du):
        """sum_m du_m^T H_m du_m."""
        return float(sum(du[m] @ (self.H[m] @ du[m]) for m in range(self.M)))

    def spread(self, u0, w0_sites):
        M, S = self.M, self.model.S
        I0, R0 = self.model.reaction(u0, w0_sites, np.arange(S))
        return {"u0": u0.copy(), "w0": w0_sites.copy(), "u": np.tile(u0, (M, 1)),
                "w": np.tile(w0_sites, (M, 1)), "I": np.tile(I0, (M, 1)), "R": np.tile(R0, (M, 1))}

    def _solve(self, m, rhs, idx):
        if not self.direct:
            return jacobi_pcg(self.H[m], rhs, idx, self.cg_rtol, self.cg_maxit)
        x = np.zeros(self.model.N)
        if idx.size:
            x[idx] = splu(self.H[m][idx][:, idx].tocsc()).solve(rhs[idx])
        return x, 0

    def sweep(self, st, idx):
        """One sweep on nodes idx (ascending); returns (next idx, info)."""
        M, dt = self.M, self.dt
        Q, QI, QE = self.col.Q, self.col.QI, self.col.QE
        mod = self.model
        A, Mm, N, S = mod.A, mod.M, mod.N, mod.S
        u, w, I, R = st["u"], st["w"], st["I"], st["R"]
        u0, w0 = st["u0"], st["w0"]
        active = np.zeros(N, dtype=bool)
        active[idx] = True
        sidx = np.nonzero(active[mod.si])[0]          # sites whose intracellular node is active

        F = np.zeros((M, N))
        for j in range(M):
            F[j, idx] = -(A @ u[j])[idx] - mod.bvec(I[j])[idx]
        Phi = np.zeros((M, N))
        Gam = np.zeros((M, S))
        for m in range(M):
            Phi[m, idx] = (Mm @ (u0 - u[m]))[idx] + dt * (Q[m, :] @ F[:, idx])
            Gam[m, sidx] = w0[sidx] - w[m, sidx] + dt * (Q[m, :] @ R[:, sidx])

        du = np.zeros((M, N))
        dI = np.zeros((M, S))
        dR = np.zeros((M, S))
        amax = np.zeros(N)
        iters = []
        for m in range(M):
            dw = Gam[m, sidx].copy()
            rhs = np.zeros(N)
            rhs[idx] = Phi[m, idx]
            y = np.zeros(N)
            for j in range(m):
                dw += dt * QE[m, j] * dR[j, sidx]
                rhs[idx] -= dt * QE[m, j] * mod.bvec(dI[j])[idx]
                y += dt * QI[m, j] * du[j]
            rhs[idx] -= (A @ y)[idx]
            x, it = self._solve(m, rhs, idx)
            iters.append(it)
            du[m] = x
            u[m, idx] += x[idx]
            w[m, sidx] += dw
            In, Rn = mod.reaction(u[m], w[m, sidx], sidx)
            dI[m, sidx] = In - I[m, sidx]
            dR[m, sidx] = Rn - R[m, sidx]
            I[m, sidx] = In
            R[m, sidx] = Rn
            amax[idx] = np.maximum(amax[idx], np.abs(x[idx]))
        if self.theta <= 0.0:
            nxt = idx.copy()
        else:
            nxt = idx[amax[idx] >= self.theta]
        return nxt, {"n_active": int(idx.size), "cg_iters": iters, "amax": amax, "du": du}

    def step(self, u0, w0_sites, K, idx_replay=None):
        st = self.spread(u0, w0_sites)
        idx = np.arange(self.model.N)
        infos = []
        thr = ((1.0 - self.rho) / self.rho * self.tol_sdc) ** 2
        for k in range(K):
            if idx_replay is not None and k > 0 and idx_replay[k] is not None:
                idx = np.asarray(idx_replay[k], dtype=np.int64)
            idx, info = self.sweep(st, idx)
            infos.append(info)
            if self.tol_sdc > 0.0:
                info["energy"] = self.energy(info["du"])
                if k + 1 >= self.K_min and info["energy"] <= thr:
                    break
        return st["u"][-1].copy(), st["w"][-1].copy(), infos


def build(P, direct=False, tol_sdc=0.0, rho=0.05, K_min=1):
    return EmiSDC(EMI(P), P.M, P.dt, P.theta, P.cg_rtol, P.cg_maxit, direct=direct, tol_sdc=tol_sdc, rho=rho,
                  K_min=K_min)


def run(sdc, u, w_sites, n_steps, K, stimuli=(), t0=0.0, idx_replay=None):
    """n_steps steps; stimuli overwrite u on their nodes at the start of the step that contains them."""
    u = np.array(u, dtype=np.float64)
    w = np.array(w_sites, dtype=np.float64)
    log = []
    for n in range(n_steps):
        t = t0 + n * sdc.dt
        apply_stimuli(u, t, sdc.dt, stimuli)
        u, w, infos = sdc.step(u, w, K, None if idx_replay is None else idx_replay[n])
        log.append(infos)
    return u, w, log


def collocation_solution(model, M, dt, u0, w0_sites):
    """The Radau-IIA collocation solution of one step (Sec. 3.1): the stage
    values (u_m, w_m) with M (u_m - u0) = dt sum_j Q[m,j] (-A u_j - b_j) and
    w_m - w0 = dt sum_j Q[m,j] R_j, solved by Newton's method with the exact
    Jacobian and dense LU (tiny meshes only)."""
    col = Collocation(M)
    Q = col.Q
    N, S = model.N, model.S
    A = model.A.toarray()
    Mm = model.M.toarray()
    si, se, l = model.si, model.se, model.l
    Ev = np.zeros((S, N))                     # v = Ev u
    Ev[np.arange(S), si] = 1.0
    Ev[np.arange(S), se] = -1.0
    Bt = (Ev * l[:, None]).T                  # b = Bt I
    p = model.p
    z = np.concatenate([np.tile(u0, M), np.tile(w0_sites, M)])
    for _ in range(60):
        U = z[:M * N].reshape(M, N)
        W = z[M * N:].reshape(M, S)
        V = U @ Ev.T
        I = ionic.current(V, W, p)
        Rr = ionic.rate(V, W, p)
        Iv, Iw, _ = ionic.current_partials(V, W, p)
        Rv, Rw, _ = ionic.rate_partials(V, W, p)
        res_u = np.stack([Mm @ (U[m] - u0) - dt * sum(Q[m, j] * (-A @ U[j] - Bt @ I[j]) for j in range(M))
                          for m in range(M)])
        res_w = np.stack([W[m] - w0_sites - dt * sum(Q[m, j] * Rr[j] for j in range(M)) for m in range(M)])
        res = np.concatenate([res_u.ravel(), res_w.ravel()])
        J = np.zeros((M * (N + S), M * (N + S)))
        for m in range(M):
            ru = slice(m * N, (m + 1) * N)
            rw = slice(M * N + m * S, M * N + (m + 1) * S)
            J[ru, ru] += Mm
            J[rw, rw] += np.eye(S)
            for j in range(M):
                cu = slice(j * N, (j + 1) * N)
                cw = slice(M * N + j * S, M * N + (j + 1) * S)
                J[ru, cu] += dt * Q[m, j] * (A + Bt @ (Iv[j][:, None] * Ev))
                J[ru, cw] += dt * Q[m, j] * (Bt * Iw[j][None, :])
                J[rw, cu] -= dt * Q[m, j] * (Rv[j][:, None] * Ev)
                J[rw, cw] -= dt * Q[m, j] * np.diag(Rw[j])
        dz = np.linalg.solve(J, -res)
        z = z + dz
        if np.max(np.abs(dz)) <= 1e-15 * max(1.0, np.max(np.abs(z))):
            break
    return z[:M * N].reshape(M, N), z[M * N:].reshape(M, S)
