"""Python binding of the adaptive SDC library: argument marshalling only.

Device memory and streams come from PyTorch (HIP build); every step of the
method runs in the HIP library.  Tensors passed in must be contiguous and on
the solver's device: float64 for values, int32 for index lists.
"""
import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import MAX_NODES, MAX_SWEEPS, Params, StepStats, SweepStats  # noqa: F401


class SDCError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_lib.ERRORS.get(code, code)}: {msg}")
        self.code = code


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _host(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(ctypes.c_void_p)


def collocation(M):
    """(tau, Q, QI, QE) as computed by the library (host call)."""
    lib = _lib.load()
    out = [np.zeros(M), np.zeros((M, M)), np.zeros((M, M)), np.zeros((M, M))]
    rc = lib.sdc_collocation(M, *[o.ctypes.data_as(ctypes.c_void_p) for o in out])
    if rc != 0:
        raise SDCError(rc, "sdc_collocation")
    return tuple(out)


def select_noalloc(amax, idx, theta, idx_out, n_out, stream=None):
    """Allocation-free compaction (sdc_select_noalloc): writes the entries i
    of idx with amax[i] >= theta to idx_out and their count to n_out[0] (-1
    when an entry lies outside amax), on the given stream, without
    allocating or synchronising.  amax float64, idx and idx_out int32 (room
    for idx.numel() entries), n_out int64 [1]: contiguous tensors on one
    device."""
    lib = _lib.load()
    dev = amax.device
    for t, dt in ((amax, torch.float64), (idx, torch.int32), (idx_out, torch.int32), (n_out, torch.int64)):
        if t.device != dev or t.dtype != dt or not t.is_contiguous():
            raise ValueError(f"expected a contiguous {dt} tensor on {dev}")
    if idx_out.numel() < idx.numel() or n_out.numel() < 1:
        raise ValueError("idx_out needs room for every entry of idx, n_out one entry")
    if idx.numel() > _lib.NOALLOC_MAX_IN:
        raise ValueError(f"at most {_lib.NOALLOC_MAX_IN} entries (the library's fixed scratch)")
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    rc = lib.sdc_select_noalloc(dev.index, ctypes.c_void_p(st.cuda_stream), _ptr(amax), amax.numel(), _ptr(idx),
                                idx.numel(), float(theta), _ptr(idx_out), _ptr(n_out))
    if rc != 0:
        raise SDCError(rc, "sdc_select_noalloc: bad arguments (sizes, pointers, device)" if rc == -1 else
                       "sdc_select_noalloc: launch failed")


class Solver:
    """One library context: an assembled mesh (possibly several instances)."""

    def __init__(self, coords, elems, elem_tensor, node_sigma, ionic, node_off, elem_off,
                 M, K, dt, theta, cg_rtol=1e-12, cg_maxit=1000, fmt=0, device=None, stream=None, emi=None,
                 tol_sdc=0.0, rho=0.05, K_min=1, drop="theta", scheme="imex", first_rings=0,
                 first_full_every=10, small_set_rows=0, rows_per_thread=0, cg_energy_tol=0.0, cg_delay=4):
        """emi: None (monodomain) or a dict with the cell-by-cell couplings
        mem_intra, mem_extra, mem_len, cm, gap_a, gap_b, gap_len, g_gap,
        robin_len, eps (see sdc_emi).  drop: "theta" (fixed drop tolerance)
        or "apriori" (per instance and step from tol_sdc and rho, see
        sdc_params.drop_mode).  scheme: "imex" (explicit reaction) or
        "linearized" (the paper's basic scheme, see sdc_params.scheme).
        first_rings >= 1: heuristic first-sweep sets grown by that many rings
        of mesh neighbours, with all rows every first_full_every steps (see
        sdc_params.first_rings).  small_set_rows: solves of at most that many
        rows per instance run in one launch each (0: up to 2048, 1024 when rows
        hold more than 8 entries; -1: never).  rows_per_thread: all-rows CG
        launches with diagonal storage take 1 or 2 rows per thread (0: the
        faster, timed at setup).  cg_energy_tol > 0: every CG solve also stops
        at that estimated relative energy error, estimated over cg_delay
        steps (see sdc_params.cg_energy_tol; 1e-3 is the paper's value)."""
        if drop not in ("theta", "apriori"):
            raise ValueError("drop must be 'theta' or 'apriori'")
        if scheme not in ("imex", "linearized"):
            raise ValueError("scheme must be 'imex' or 'linearized'")
        self.lib = _lib.load()
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        ctx = ctypes.c_void_p()
        rc = self.lib.sdc_create(ctypes.byref(ctx), self.device.index, ctypes.c_void_p(stream.cuda_stream))
        if rc != 0:
            raise SDCError(rc, "sdc_create failed")
        self.ctx = ctx
        coords = np.asarray(coords, dtype=np.float64)
        dim = coords.shape[1]
        self.M, self.K = int(M), int(K)
        prm = Params(M=self.M, K=self.K, dt=float(dt), theta=float(theta), cg_rtol=float(cg_rtol),
                     cg_maxit=int(cg_maxit), format=int(fmt), K_min=int(K_min), tol_sdc=float(tol_sdc),
                     rho=float(rho), drop_mode=1 if drop == "apriori" else 0,
                     scheme=1 if scheme == "linearized" else 0, first_rings=int(first_rings),
                     first_full_every=int(first_full_every), small_set_rows=int(small_set_rows),
                     rows_per_thread=int(rows_per_thread), cg_energy_tol=float(cg_energy_tol),
                     cg_delay=int(cg_delay))
        node_off_a, p_no = _host(node_off, np.int64)
        coords_a, p_c = _host(coords, np.float64)
        elem_off_a, p_eo = _host(elem_off, np.int64)
        elems_a, p_e = _host(elems, np.int32)
        tens_a, p_t = _host(elem_tensor, np.float64)
        sig_a, p_s = _host(node_sigma, np.float64)
        ion_a, p_i = _host(np.atleast_2d(ionic), np.float64)
        emi_arg = None
        if emi is not None:
            keep = []

            def arr(x, dt):
                a, ptr = _host(x, dt)
                keep.append(a)
                return ptr.value

            emi_arg = _lib.Emi(n_mem=len(emi["mem_intra"]), mem_intra=arr(emi["mem_intra"], np.int32),
                               mem_extra=arr(emi["mem_extra"], np.int32), mem_len=arr(emi["mem_len"], np.float64),
                               cm=float(emi["cm"]), n_gap=len(emi["gap_a"]), gap_a=arr(emi["gap_a"], np.int32),
                               gap_b=arr(emi["gap_b"], np.int32), gap_len=arr(emi["gap_len"], np.float64),
                               g_gap=float(emi["g_gap"]), robin_len=arr(emi["robin_len"], np.float64),
                               eps=float(emi["eps"]))
        self._check(self.lib.sdc_setup_mesh(self.ctx, ctypes.byref(prm), dim, len(node_off_a) - 1,
                                            p_no, p_c, p_eo, p_e, p_t, p_s, p_i,
                                            ctypes.byref(emi_arg) if emi_arg is not None else None))
        self.emi = emi is not None
        n, nnz, nw = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        self._check(self.lib.sdc_get_sizes(self.ctx, ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(nw)))
        self.N, self.nnz, self.Nw = n.value, nnz.value, nw.value
        self.n_inst = len(node_off_a) - 1
        self.dt = float(dt)
        self.ionic = ion_a.copy()
        self.node_sigma = sig_a.copy()
        self.max_recordings = _lib.MAX_RECORDINGS

    @classmethod
    def from_problem(cls, P, **kw):
        """Context for a workloads.Problem, with its stimuli registered."""
        args = dict(M=P.M, K=P.K, dt=P.dt, theta=P.theta, cg_rtol=P.cg_rtol, cg_maxit=P.cg_maxit)
        if hasattr(P, "mem_intra"):   # cell-by-cell problem
            args["emi"] = {k: getattr(P, k) for k in ("mem_intra", "mem_extra", "mem_len", "cm", "gap_a", "gap_b",
                                                      "gap_len", "g_gap", "robin_len", "eps")}
        args.update(kw)
        s = cls(P.coords, P.elems, P.elem_tensor, P.node_sigma, P.ionic, P.node_off, P.elem_off, **args)
        for t_on, nodes, value in P.stimuli:
            s.add_stimulus(t_on, nodes, value)
        return s

    # -- plumbing ---------------------------------------------------------
    def _check(self, rc):
        if rc != 0:
            msg = self.lib.sdc_last_error(self.ctx)
            raise SDCError(rc, msg.decode() if msg else "")

    def _vec(self, t, dtype=torch.float64, n=None):
        if not isinstance(t, torch.Tensor) or t.device != self.device or t.dtype != dtype or not t.is_contiguous():
            raise ValueError(f"expected a contiguous {dtype} tensor on {self.device}")
        if n is not None and t.numel() < n:
            raise ValueError(f"tensor too small: {t.numel()} < {n}")
        return _ptr(t)

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.sdc_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- API --------------------------------------------------------------
    def add_stimulus(self, t_on, nodes, value):
        a, p = _host(nodes, np.int32)
        self._check(self.lib.sdc_add_stimulus(self.ctx, float(t_on), p, a.size, float(value)))

    def system(self):
        """(rowptr, col, val, ml) of the assembled A and lumped mass (numpy)."""
        rp = np.zeros(self.N + 1, np.int32)
        col = np.zeros(self.nnz, np.int32)
        val = np.zeros(self.nnz)
        ml = np.zeros(self.N)
        self._check(self.lib.sdc_get_system(self.ctx, *[x.ctypes.data_as(ctypes.c_void_p) for x in (rp, col, val, ml)]))
        return rp, col, val, ml

    def step(self, v, w, t, stats=False):
        """Advance (v, w) in place by one step from time t."""
        st = StepStats() if stats else None
        self._check(self.lib.sdc_step(self.ctx, self._vec(v, n=self.N), self._vec(w, n=self.Nw), float(t),
                                      ctypes.byref(st) if st is not None else None))
        if st is not None:
            return [st.sweep[k].as_dict(self.M) for k in range(st.n_sweeps)]
        return None

    def begin_step(self, v, w, t):
        self._check(self.lib.sdc_begin_step(self.ctx, self._vec(v, n=self.N), self._vec(w, n=self.Nw), float(t)))

    def sweep(self):
        st = SweepStats()
        self._check(self.lib.sdc_sweep(self.ctx, ctypes.byref(st)))
        return st.as_dict(self.M)

    def end_step(self, v, w):
        self._check(self.lib.sdc_end_step(self.ctx, self._vec(v, n=self.N), self._vec(w, n=self.Nw)))

    def node(self, m):
        v = torch.empty(self.N, dtype=torch.float64, device=self.device)
        w = torch.empty(self.Nw, dtype=torch.float64, device=self.device)
        self._check(self.lib.sdc_get_node(self.ctx, int(m), _ptr(v), _ptr(w)))
        return v, w

    def cg_iters(self):
        """CG updates of the last sweep's solves: int array [M, n_inst]."""
        out = np.zeros((self.M, self.n_inst), dtype=np.int32)
        self._check(self.lib.sdc_get_cg_iters(self.ctx, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def active(self):
        n = ctypes.c_int64()
        self._check(self.lib.sdc_get_active(self.ctx, None, ctypes.byref(n)))
        idx = torch.empty(max(self.N, 1), dtype=torch.int32, device=self.device)
        self._check(self.lib.sdc_get_active(self.ctx, _ptr(idx), ctypes.byref(n)))
        return idx[: n.value].clone()

    def set_active(self, sweep, idx):
        """Pin the set of sweep `sweep` (>= 1); idx=None clears every pin."""
        if idx is None:
            self._check(self.lib.sdc_set_active(self.ctx, -1, None, 0))
            return
        self._check(self.lib.sdc_set_active(self.ctx, int(sweep), self._vec(idx, torch.int32), idx.numel()))

    def solve(self, m, idx, b):
        x = torch.empty(self.N, dtype=torch.float64, device=self.device)
        iters = (ctypes.c_int32 * self.n_inst)()
        self._check(self.lib.sdc_solve(self.ctx, int(m), self._vec(idx, torch.int32), idx.numel(),
                                       self._vec(b, n=self.N), _ptr(x), iters))
        return x, list(iters)

    def adjoint_step(self, v_n, w_n, t, lam_v, lam_w, g_sigma, g_a):
        """Reverse of step(v_n, w_n, t): lam_v, lam_w updated in place to the
        adjoints of (v_n, w_n); the sensitivities are added to g_sigma [N]
        and g_a [n_inst]."""
        self._check(self.lib.sdc_adjoint_step(
            self.ctx, self._vec(v_n, n=self.N), self._vec(w_n, n=self.Nw), float(t), self._vec(lam_v, n=self.N),
            self._vec(lam_w, n=self.Nw), self._vec(g_sigma, n=self.N), self._vec(g_a, n=self.n_inst)))

    def adjoint_record(self, slot, v, w, t):
        """Advance (v, w) in place by one step from t, recording it in `slot` for adjoint_reverse."""
        self._check(self.lib.sdc_adjoint_record(self.ctx, int(slot), self._vec(v, n=self.N),
                                                self._vec(w, n=self.Nw), float(t)))

    def adjoint_reverse(self, slot, lam_v, lam_w, g_sigma, g_a):
        """Reverse step of recording `slot` (see adjoint_step)."""
        self._check(self.lib.sdc_adjoint_reverse(self.ctx, int(slot), self._vec(lam_v, n=self.N),
                                                 self._vec(lam_w, n=self.Nw), self._vec(g_sigma, n=self.N),
                                                 self._vec(g_a, n=self.n_inst)))

    def set_coefficients(self, node_sigma=None, ionic=None):
        """Reassemble with new nodal conductivity multipliers and/or ionic parameters (host arrays)."""
        ps = pi = None
        if node_sigma is not None:
            s_a, ps = _host(node_sigma, np.float64)
            assert s_a.size == self.N
        if ionic is not None:
            i_a, pi = _host(np.atleast_2d(ionic), np.float64)
            assert i_a.shape == (self.n_inst, 6)
        self._check(self.lib.sdc_set_coefficients(self.ctx, ps, pi))
        if ionic is not None:
            self.ionic = i_a.copy()
        if node_sigma is not None:
            self.node_sigma = s_a.copy()

    def info(self):
        """Storage in use ('csr', 'dia' or 'sell'), diagonals, setup timings,
        redone steps, rows per thread of the all-rows CG launches and their
        timings, graph-mode counts, and the XCD chunk of the work maps (blocks
        of 256 rows; 0 = contiguous eighths)."""
        st = _lib.Info()
        self._check(self.lib.sdc_get_info(self.ctx, ctypes.byref(st)))
        return {"format": {1: "csr", 2: "dia", 3: "sell"}[st.format], "n_diagonals": st.n_diagonals,
                "t_csr_us": st.t_csr_us, "t_dia_us": st.t_dia_us, "redone_steps": st.redone_steps,
                "rows_per_thread": st.rows_per_thread, "t_rows1_us": st.t_rows1_us, "t_rows2_us": st.t_rows2_us,
                "graph_steps": st.graph_steps, "graph_captures": st.graph_captures, "graph_redone": st.graph_redone,
                "t_sell_us": st.t_sell_us, "xcd_chunk": st.xcd_chunk}

    def set_graph(self, enable=True):
        """Graph-captured sweeps for step() (see sdc_set_graph)."""
        self._check(self.lib.sdc_set_graph(self.ctx, 1 if enable else 0))

    def profile(self, enable):
        """Start (and clear) or stop event timing of the CG kernels."""
        self._check(self.lib.sdc_profile(self.ctx, 1 if enable else 0))

    def profile_read(self):
        st = _lib.ProfileStats()
        self._check(self.lib.sdc_profile_read(self.ctx, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in st._fields_}

    def drop_tolerance(self):
        """The current step's a-priori drop tolerance per instance: a dict of
        arrays TOL_drop, r, c, eta (drop="apriori" only)."""
        out = np.zeros(4 * self.n_inst)
        self._check(self.lib.sdc_get_drop_tolerance(self.ctx, out.ctypes.data_as(ctypes.c_void_p)))
        out = out.reshape(self.n_inst, 4)
        return {"tol_drop": out[:, 0].copy(), "r": out[:, 1].astype(np.int64), "c": out[:, 2].copy(),
                "eta": out[:, 3].copy()}

    def select(self, amax, idx, theta):
        out = torch.empty(max(idx.numel(), 1), dtype=torch.int32, device=self.device)
        n = ctypes.c_int64()
        self._check(self.lib.sdc_select(self.ctx, self._vec(amax, n=self.N), self._vec(idx, torch.int32),
                                        idx.numel(), float(theta), _ptr(out), ctypes.byref(n)))
        return out[: n.value].clone()
