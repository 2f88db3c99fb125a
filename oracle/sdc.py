"""Adaptive IMEX SDC step for the monodomain system (oracle; test infrastructure).

Problem (Sec. 2.2, eq. abstract monodomain, with beta*C_m = 1 and nodal
quadrature of the reaction):

    ML v' = -A v - ML * I(v, w),      w' = R(v, w).

Time stepping (Sec. 3, eq. final-sdc).  We follow the implicit-explicit
reading: diffusion implicit through the lower-triangular QI (LU trick),
reaction and gating explicit through QE (forward Euler between nodes); the
paper's lumped reaction Jacobian on the diagonal of the system matrix is not
used, so every solve has the matrix H_m = ML + dt*QI[m,m]*A.  In Q form, one
sweep over nodes m = 0..M-1 reads

    Phi_m  = ML (v0 - v_m) + dt sum_j Q[m,j] (-A v_j - ML I_j)
    Gam_m  = w0 - w_m + dt sum_j Q[m,j] R_j
    dw_m   = Gam_m + dt sum_{j<m} QE[m,j] dR_j
    H_m dv_m = Phi_m - dt sum_{j<m} QE[m,j] ML dI_j - A (dt sum_{j<m} QI[m,j] dv_j)
    v_m += dv_m,  w_m += dw_m,  (I_m, R_m) <- AP(v_m, w_m),
    dI_m, dR_m = change of I_m, R_m in this sweep.

Algebraic adaptivity (Sec. 4.2): sweep k only touches the rows of the index
set I_k; its solves use the principal submatrix H_m[I_k, I_k] (zero
correction on the complement); rows outside I_k keep the values they have.
The next set keeps the rows whose correction reached the drop tolerance,

    I_{k+1} = { i in I_k : max_m |dv_m,i| >= theta },

so the sets are nested.  Readings: the maximum over collocation nodes is
taken (the bound of Thm. 1 is in L-infinity over the step); the gating
correction does not enter the rule; theta <= 0 keeps every row (the
non-adaptive method); every step starts with all rows active and with the
collocation values spread from the step's initial state.

Optionally (``run(..., first=FirstSweepSubset(...))``) a step's first sweep
takes a heuristic a-priori set instead of all rows; the paper names such a
subset (Sec. 6) without fixing a rule, and the one here is a reading: the
set the previous step carried after its first sweep and this step's
stimulated rows, grown by rings of mesh neighbours, with a full first sweep
on the run's first step and on every full_every-th step.  Rows outside the
set keep their spread values (no change over the step).
"""
import numpy as np
import scipy.sparse as sp

from . import ionic
from .collocation import Collocation
from .pcg import jacobi_pcg


class Monodomain:
    """ML, A and per-node ionic parameters of a (possibly multi-instance) mesh.

    ``ionic_params`` has shape [N, 6]: one Aliev-Panfilov parameter set per
    node, so that several instances with different parameters can share one
    vector layout.
    """

    def __init__(self, ML, A, ionic_params):
        self.ML = np.asarray(ML, dtype=np.float64)
        self.A = A.tocsr()
        self.N = self.ML.size
        p = np.asarray(ionic_params, dtype=np.float64)
        if p.ndim == 1:
            p = np.broadcast_to(p, (self.N, 6))
        self.p = p.T.copy()          # [6, N] so ionic.current(v, w, p) broadcasts

    def reaction(self, v, w, rows):
        p = self.p[:, rows]
        return ionic.current(v, w, p), ionic.rate(v, w, p)


def sweeps_needed(c, rho, tol, cap=10000):
    """Smallest integer r >= 0 with c rho^r <= (1 - rho) tol: the iteration
    count of Thm. 2 (eq. r-condition, r >= log((1-rho) TOL / c) / log rho),
    found by repeated multiplication so that the integer is decided by the
    same floating-point products wherever it is computed."""
    bound = (1.0 - rho) * tol
    r, q = 0, float(c)
    while q > bound and r < cap:
        q *= rho
        r += 1
    return r


def apriori_drop_tolerance(c, eta, dt, rho, tol):
    """Eq. drop-tolerance: TOL_drop = exp(-eta T) (1 - rho) / (r + 1) TOL over
    a step of length T = dt, with r from Thm. 2 for the correction size c."""
    r = sweeps_needed(c, rho, tol)
    return np.exp(-eta * dt) * (1.0 - rho) / (r + 1) * tol, r


class SDC:
    """IMEX SDC on Radau-IIA nodes with nested active index sets.

    Optional energy-norm termination (Sec. 3.2): with tol_sdc > 0, an
    instance stops sweeping once, after at least K_min sweeps,

        sum_m dv_m^T H_m dv_m  <=  ((1 - rho) / rho * tol_sdc)^2,

    the energy norm of the sweep's corrections with the system matrices
    H_m (reading: the paper's lumped reaction Jacobian is not part of H_m, as
    in the sweep itself).  A stopped instance's rows leave the active set;
    the step ends when every instance has stopped or after K sweeps.
    ``inst_of`` maps rows to instances (default: one instance).

    A-priori drop tolerance (``drop="apriori"``, Sec. 4.1): instead of the
    fixed theta, each instance's sets after the first sweep use
    TOL_drop = exp(-eta dt) (1 - rho) / (r + 1) tol_sdc (eq.
    drop-tolerance), with the error constant c estimated from the first
    sweep as the instance's largest correction max |dv| (rho taken as
    known, as the paper suggests), r from Thm. 2, and
    eta = max(0, -min dI/dv) / (beta C_m) (Thm. 1, beta C_m = 1) over the
    instance's rows at the step's start state and at the collocation
    values after the first sweep.
    """

    def __init__(self, model, M, dt, theta, cg_rtol=1e-12, cg_maxit=1000, tol_sdc=0.0, rho=0.05, K_min=1,
                 inst_of=None, drop="theta", scheme="imex", cg_energy_tol=0.0, cg_delay=0):
        self.model = model
        self.col = Collocation(M)
        self.M = M
        self.dt = float(dt)
        self.theta = float(theta)
        self.cg_rtol = cg_rtol
        self.cg_maxit = cg_maxit
        # optional energy-error stop of every solve (see jacobi_pcg)
        self.cg_energy_tol = float(cg_energy_tol)
        self.cg_delay = int(cg_delay)
        self.tol_sdc = float(tol_sdc)
        self.rho = float(rho)
        self.K_min = int(K_min)
        if drop not in ("theta", "apriori"):
            raise ValueError("drop must be 'theta' or 'apriori'")
        if drop == "apriori" and not (self.tol_sdc > 0.0 and 0.0 < self.rho < 1.0):
            raise ValueError("the a-priori drop tolerance needs tol_sdc > 0 and 0 < rho < 1")
        self.drop = drop
        if scheme not in ("imex", "linearized"):
            raise ValueError("scheme must be 'imex' or 'linearized'")
        self.scheme = scheme
        self._Hk = None   # the linearized scheme's system matrices of the last sweep
        self.inst_of = np.zeros(model.N, dtype=np.int64) if inst_of is None else np.asarray(inst_of, dtype=np.int64)
        self.n_inst = int(self.inst_of.max()) + 1 if self.inst_of.size else 1
        ML, A = model.ML, model.A
        self.H = [(sp.diags(ML) + self.dt * self.col.QI[m, m] * A).tocsr() for m in range(M)]

    def energy(self, dv):
        """Per instance: sum_m dv_m^T H_m dv_m (the last sweep's matrices in
        the linearized scheme)."""
        H = self._Hk if self.scheme == "linearized" else self.H
        e = np.zeros(self.n_inst)
        for m in range(self.M):
            np.add.at(e, self.inst_of, dv[m] * (H[m] @ dv[m]))
        return e

    # -- one step -------------------------------------------------------
    def spread(self, v0, w0):
        """Initial guess: every collocation value equals the step's start value."""
        M, N = self.M, self.model.N
        st = {
            "v0": v0.copy(), "w0": w0.copy(),
            "v": np.tile(v0, (M, 1)), "w": np.tile(w0, (M, 1)),
        }
        I0, R0 = self.model.reaction(v0, w0, np.arange(N))
        st["I"] = np.tile(I0, (M, 1))
        st["R"] = np.tile(R0, (M, 1))
        return st

    def drop_tolerances(self, st, amax, idx):
        """Per instance (TOL_drop, r, c, eta) after the first sweep on idx."""
        n = self.n_inst
        c = np.zeros(n)
        np.maximum.at(c, self.inst_of[idx], amax[idx])
        p = self.model.p[:, idx]
        dmin = np.full(n, np.inf)
        states = [(st["v0"][idx], st["w0"][idx])] + [(st["v"][m, idx], st["w"][m, idx]) for m in range(self.M)]
        for v, w in states:
            np.minimum.at(dmin, self.inst_of[idx], ionic.current_partials(v, w, p)[0])
        eta = np.maximum(0.0, -dmin)
        eta[~np.isfinite(eta)] = 0.0   # an instance without rows
        out = [apriori_drop_tolerance(c[i], eta[i], self.dt, self.rho, self.tol_sdc) for i in range(n)]
        return np.array([o[0] for o in out]), np.array([o[1] for o in out]), c, eta

    def sweep(self, st, idx, cg_iters=None, theta=None):
        """One sweep on rows idx (ascending int array); returns (next idx, info).
        theta: the drop tolerance (default self.theta), or one per instance."""
        M, dt = self.M, self.dt
        Q, QI, QE = self.col.Q, self.col.QI, self.col.QE
        ML, A = self.model.ML, self.model.A
        N = self.model.N
        v, w, I, R = st["v"], st["w"], st["I"], st["R"]
        v0, w0 = st["v0"], st["w0"]

        # sweep-start residuals on the active rows (full rows of A)
        F = np.zeros((M, N))
        for j in range(M):
            F[j, idx] = -(A @ v[j])[idx] - ML[idx] * I[j, idx]
        Phi = np.zeros((M, N))
        Gam = np.zeros((M, N))
        for m in range(M):
            Phi[m, idx] = ML[idx] * (v0[idx] - v[m, idx]) + dt * (Q[m, :] @ F[:, idx])
            Gam[m, idx] = w0[idx] - w[m, idx] + dt * (Q[m, :] @ R[:, idx])

        if self.scheme == "linearized":
            dv, amax, iters = self._solve_linearized(st, idx, Phi, cg_iters)
        else:
            dv, amax, iters = self._solve_imex(st, idx, Phi, Gam, cg_iters)
        if theta is None or np.ndim(theta) == 0:
            nxt = select(idx, amax, self.theta if theta is None else float(theta))
        else:
            nxt = idx[amax[idx] >= np.asarray(theta)[self.inst_of[idx]]]
        # per node: the largest step count over instances, and every instance's
        return nxt, {"idx": idx, "n_active": int(idx.size), "cg_iters": [int(np.max(it)) for it in iters],
                     "cg_iters_inst": [np.asarray(it).copy() for it in iters], "amax": amax, "dv": dv}

    def _pcg(self, H, b, idx, fixed):
        """The restricted solve of one node.  The instances are independent
        systems, so each is solved by a CG of its own (its own scalars and
        stopping test).  Returns x and the per-instance step counts; `fixed`
        replays counts, one per instance or one for all."""
        x = np.zeros(H.shape[0])
        its = np.zeros(self.n_inst, dtype=np.int64)
        log = getattr(self, "solve_log", None)   # a list: record (H, b, rows, steps) of every solve
        if fixed is not None:
            fixed = np.broadcast_to(np.asarray(fixed, dtype=np.int64).reshape(-1), (self.n_inst,))
        for i in range(self.n_inst):
            sub = idx if self.n_inst == 1 else idx[self.inst_of[idx] == i]
            fi = None if fixed is None else int(fixed[i])
            xi, its[i] = jacobi_pcg(H, b, sub, self.cg_rtol, self.cg_maxit, fi, self.cg_energy_tol, self.cg_delay)
            x[sub] = xi[sub]
            if log is not None:
                log.append((H, b, sub, int(its[i])))
        return x, its

    def _solve_imex(self, st, idx, Phi, Gam, cg_iters):
        """Node by node: implicit diffusion, explicit reaction and gating."""
        M, dt = self.M, self.dt
        QI, QE = self.col.QI, self.col.QE
        ML, A = self.model.ML, self.model.A
        N = self.model.N
        v, w, I, R = st["v"], st["w"], st["I"], st["R"]
        dv = np.zeros((M, N))
        dI = np.zeros((M, N))
        dR = np.zeros((M, N))
        amax = np.zeros(N)
        iters = []
        for m in range(M):
            dw = Gam[m, idx].copy()
            rhs = Phi[m, idx].copy()
            y = np.zeros(N)
            for j in range(m):
                dw += dt * QE[m, j] * dR[j, idx]
                rhs -= dt * QE[m, j] * ML[idx] * dI[j, idx]
                y += dt * QI[m, j] * dv[j]
            rhs -= (A @ y)[idx]
            b = np.zeros(N)
            b[idx] = rhs
            fixed = None if cg_iters is None else cg_iters[m]
            x, it = self._pcg(self.H[m], b, idx, fixed)
            iters.append(it)
            dv[m] = x
            v[m, idx] += x[idx]
            w[m, idx] += dw
            In, Rn = self.model.reaction(v[m, idx], w[m, idx], idx)
            dI[m, idx] = In - I[m, idx]
            dR[m, idx] = Rn - R[m, idx]
            I[m, idx] = In
            R[m, idx] = Rn
            amax[idx] = np.maximum(amax[idx], np.abs(x[idx]))
        return dv, amax, iters

    def _solve_linearized(self, st, idx, Phi, cg_iters):
        """The paper's basic scheme (eq. final-sdc): per node, the potential
        correction with the lumped reaction Jacobian G_j = ML dI/dv(v_j, w_j)
        (at the sweep's iterate) beside A in the LU-trick operator,

            (ML + dt QI[m,m] (A + G_m)) dv_m = Phi_m - dt sum_{j<m} QI[m,j] (A + G_j) dv_j,

        then, with the new potentials, the gating correction with the
        implicit dR/dw (Gauss-Seidel, u then w):

            (1 - dt QI[m,m] R'_m) dw_m = w0 - w_m + dt sum_j Q[m,j] R(v_j^new, w_j)
                                         + dt sum_{j<m} QI[m,j] R'_j dw_j,
            R'_j = dR/dw(v_j^new, w_j)."""
        M, dt = self.M, self.dt
        Q, QI = self.col.Q, self.col.QI
        ML, A = self.model.ML, self.model.A
        N = self.model.N
        v, w, I, R = st["v"], st["w"], st["I"], st["R"]
        w0 = st["w0"]
        p = self.model.p[:, idx]
        G = np.zeros((M, N))
        for j in range(M):
            G[j, idx] = ML[idx] * ionic.current_partials(v[j, idx], w[j, idx], p)[0]
        dv = np.zeros((M, N))
        amax = np.zeros(N)
        iters, Hk = [], []
        for m in range(M):
            rhs = Phi[m, idx].copy()
            y = np.zeros(N)
            for j in range(m):
                y += dt * QI[m, j] * dv[j]
                rhs -= dt * QI[m, j] * G[j, idx] * dv[j, idx]
            rhs -= (A @ y)[idx]
            Hm = (sp.diags(ML + dt * QI[m, m] * G[m]) + dt * QI[m, m] * A).tocsr()
            b = np.zeros(N)
            b[idx] = rhs
            fixed = None if cg_iters is None else cg_iters[m]
            x, it = self._pcg(Hm, b, idx, fixed)
            iters.append(it)
            Hk.append(Hm)
            dv[m] = x
            v[m, idx] += x[idx]
            amax[idx] = np.maximum(amax[idx], np.abs(x[idx]))
        Rn = [ionic.rate(v[j, idx], w[j, idx], p) for j in range(M)]
        Rw = [ionic.rate_partials(v[j, idx], w[j, idx], p)[1] for j in range(M)]
        dw = []
        for m in range(M):
            g = w0[idx] - w[m, idx] + dt * sum(Q[m, j] * Rn[j] for j in range(M))
            for j in range(m):
                g = g + dt * QI[m, j] * Rw[j] * dw[j]
            dw.append(g / (1.0 - dt * QI[m, m] * Rw[m]))
        for m in range(M):
            w[m, idx] += dw[m]
            I[m, idx], R[m, idx] = self.model.reaction(v[m, idx], w[m, idx], idx)
        self._Hk = Hk
        return dv, amax, iters

    def step(self, v0, w0, K, idx_replay=None, cg_replay=None, keep=False):
        """K sweeps from the spread state; returns (v_end, w_end, infos).

        idx_replay[k], when given, replaces the computed index set of sweep k
        (the first sweep always uses all rows unless replayed);
        cg_replay[k][m] replays CG iteration counts (one per instance, or one
        for all).
        """
        st = self.spread(v0, w0)
        idx = np.arange(self.model.N)
        infos = []
        stopped = np.zeros(self.n_inst, dtype=bool)
        theta = None
        self.carried = None
        for k in range(K):
            if idx_replay is not None and idx_replay[k] is not None:
                idx = np.asarray(idx_replay[k], dtype=np.int64)
            nxt, info = self.sweep(st, idx, None if cg_replay is None else cg_replay[k], theta)
            if self.drop == "apriori" and k == 0:
                theta, r, c, eta = self.drop_tolerances(st, info["amax"], idx)
                info.update(drop_tol=theta, drop_r=r, drop_c=c, drop_eta=eta)
                nxt = idx[info["amax"][idx] >= theta[self.inst_of[idx]]]
            if self.tol_sdc > 0.0:
                e = self.energy(info["dv"])
                info["energy"] = e
                if k + 1 >= self.K_min:
                    stopped |= e <= ((1.0 - self.rho) / self.rho * self.tol_sdc) ** 2
                nxt = nxt[~stopped[self.inst_of[nxt]]]
            if k == 0:
                # the set the step carries: that of its second sweep (its
                # first sweep's own set when the step has one sweep)
                self.carried = nxt if K > 1 else idx
                if K > 1 and idx_replay is not None and len(idx_replay) > 1 and idx_replay[1] is not None:
                    self.carried = np.asarray(idx_replay[1], dtype=np.int64)
            if not keep:
                info.pop("dv")
                info.pop("amax")
            infos.append(info)
            idx = nxt
            if stopped.all():
                break
        return st["v"][-1].copy(), st["w"][-1].copy(), infos


def mesh_adjacency(elems, N):
    """Pattern of the P1 matrices: rows i and j are adjacent when the two
    vertices share a simplex (every row is adjacent to itself)."""
    e = np.asarray(elems, dtype=np.int64)
    nv = e.shape[1]
    r = np.repeat(e, nv, axis=1).ravel()
    c = np.tile(e, (1, nv)).ravel()
    return sp.csr_matrix((np.ones(r.size), (r, c)), shape=(N, N))


def first_sweep_set(adj, carried, forced, rings):
    """Heuristic a-priori set of a step's first sweep.  The paper (Sec. 6)
    names a heuristic a-priori subset for the first sweep as a way past the
    full first sweep, which bounds the speedup, without fixing one; the rule
    here is a reading: the rows the previous step carried after its first
    sweep, with the rows a stimulus overwrote at this step's start, grown
    `rings` times by all their mesh neighbours.  Ascending rows."""
    mark = np.zeros(adj.shape[0], dtype=bool)
    mark[np.asarray(carried, dtype=np.int64)] = True
    mark[np.asarray(forced, dtype=np.int64)] = True
    for _ in range(rings):
        mark = mark | (adj @ mark.astype(np.float64) > 0.0)
    return np.nonzero(mark)[0]


class FirstSweepSubset:
    """When a step's first sweep uses the heuristic set: not on the first
    step of a run (nothing is carried yet) and not on every `full_every`-th
    step counted from it (full_every <= 0: only the first), which take all
    rows."""

    def __init__(self, adj, rings, full_every):
        if rings < 1:
            raise ValueError("rings must be >= 1")
        self.adj, self.rings, self.full_every = adj, int(rings), int(full_every)

    def rows(self, n, carried, forced):
        full = n == 0 if self.full_every <= 0 else n % self.full_every == 0
        if full or carried is None:
            return None
        return first_sweep_set(self.adj, carried, forced, self.rings)


def select(idx, amax, theta):
    """I_{k+1} = [i in idx : amax_i >= theta]; theta <= 0 keeps all rows."""
    if theta <= 0.0:
        return idx.copy()
    return idx[amax[idx] >= theta]


def stimulus_applies(t_on, t, dt):
    """Whether a stimulus at time t_on belongs to the step [t, t + dt) (a
    stimulus overwrites the state at the start of the step that contains its
    time).  Both ends of the interval are moved down by 1e-9 dt, so that a
    t_on on a step boundary belongs to the step starting there even when
    that step's t was accumulated with rounding just above it."""
    return t - 1e-9 * dt <= t_on < t + dt - 1e-9 * dt


def apply_stimuli(v, t, dt, stimuli):
    """Set v = value on the listed nodes of the stimuli of the step at t."""
    for t_on, nodes, value in stimuli:
        if stimulus_applies(t_on, t, dt):
            v[np.asarray(nodes, dtype=np.int64)] = value
    return v


def stimulus_nodes(t, dt, stimuli):
    """Node lists of the stimuli that apply at the step starting at t."""
    return [np.asarray(nodes, dtype=np.int64) for t_on, nodes, _ in stimuli if stimulus_applies(t_on, t, dt)]


def run(sdc, v, w, n_steps, K, stimuli=(), t0=0.0, idx_replay=None, cg_replay=None, first=None):
    """Advance n_steps; returns (v, w, per-step infos).  first: None (every
    first sweep on all rows) or a FirstSweepSubset; a replayed first-sweep
    set takes precedence over it."""
    v = np.array(v, dtype=np.float64)
    w = np.array(w, dtype=np.float64)
    log = []
    carried = None
    for n in range(n_steps):
        t = t0 + n * sdc.dt
        apply_stimuli(v, t, sdc.dt, stimuli)
        replay = None if idx_replay is None else idx_replay[n]
        if first is not None and (replay is None or replay[0] is None):
            forced = stimulus_nodes(t, sdc.dt, stimuli)
            rows = first.rows(n, carried, np.concatenate(forced) if forced else np.zeros(0, np.int64))
            if rows is not None:
                replay = [rows] + ([None] * (K - 1) if replay is None else list(replay[1:]))
        v, w, infos = sdc.step(v, w, K, replay, None if cg_replay is None else cg_replay[n])
        carried = sdc.carried
        log.append(infos)
    return v, w, log


def build(problem, tol_sdc=0.0, rho=0.05, K_min=1, drop="theta", scheme="imex", cg_energy_tol=0.0, cg_delay=0):
    """Assemble the oracle model and SDC integrator for a workload Problem."""
    from .assembly import lumped_mass, stiffness
    ML = lumped_mass(problem.coords, problem.elems, problem.N)
    A = stiffness(problem.coords, problem.elems, problem.elem_tensor, problem.node_sigma, problem.N)
    model = Monodomain(ML, A, problem.node_ionic())
    inst_of = np.repeat(np.arange(problem.n_inst), np.diff(problem.node_off))
    return SDC(model, problem.M, problem.dt, problem.theta, problem.cg_rtol, problem.cg_maxit,
               tol_sdc=tol_sdc, rho=rho, K_min=K_min, inst_of=inst_of, drop=drop, scheme=scheme,
               cg_energy_tol=cg_energy_tol, cg_delay=cg_delay)
