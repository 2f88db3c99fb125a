"""The synthetic workloads (seeded), as plain arrays.

Each builder returns a :class:`Problem`: mesh arrays, coefficient fields,
Aliev-Panfilov parameters per instance, stimulus schedule and the SDC
settings.  Sizes default to the full workloads; tests pass smaller sizes with
the same recipe.

Workloads (all FP64):

0  1D monodomain, 256 nodes on [0, 1] cm, D = 1e-3 cm^2/ms, v = 1 on x <= 0.05
   at t = 0, M = 3, K = 4, dt = 0.1 ms, 500 steps, CG rtol 1e-12,
   theta = 0 (non-adaptive) or 1e-6.
1  2D monodomain, 512 x 512 nodes on [0, 2]^2 cm, P1 triangles, anisotropic
   D = R(phi) diag(1.2e-3, 3e-4) R(phi)^T with a smoothed random fibre angle
   per cell (width 16 cells), v = 1 on x <= 0.1 at t = 0, M = 4, K = 4,
   dt = 0.2 ms, 1000 steps, theta = 1e-7.
2  3D monodomain, 128^3 nodes on a 1.5 cm cube, 5 tets per hex, fibres
   rotating from -60 to +60 degrees through z, two point stimuli of radius
   0.1 cm at t = 0 and t = 120 ms, M = 4, K = 4, dt = 0.25 ms, 1600 steps,
   theta = 1e-7.
4  48 independent 2D monodomain instances, side n ~ U{96..384}, isotropic
   sigma = 1e-3 exp(0.3 g) with g a smoothed Gaussian field, M = 3, K = 4,
   dt = 0.2 ms, 100 steps, theta = 1e-7.
"""
from dataclasses import dataclass, field

import numpy as np

from . import meshes

AP_PARAMS = (8.0, 0.15, 0.002, 0.2, 0.3, 0.25)   # k, a, eps0, mu1, mu2, s


@dataclass
class Problem:
    name: str
    dim: int
    coords: np.ndarray            # [N, dim] float64
    elems: np.ndarray             # [E, dim+1] int32, global node ids
    elem_tensor: np.ndarray       # [E, dim, dim] float64 unit conductivity tensors
    node_sigma: np.ndarray        # [N] float64 conductivity multiplier
    node_off: np.ndarray          # [n_inst+1] int64
    elem_off: np.ndarray          # [n_inst+1] int64
    ionic: np.ndarray             # [n_inst, 6] float64
    M: int
    K: int
    dt: float
    n_steps: int
    theta: float
    cg_rtol: float = 1e-12
    cg_maxit: int = 1000
    stimuli: list = field(default_factory=list)   # (t_on, int32 nodes, value)
    v_init: np.ndarray = None
    w_init: np.ndarray = None

    @property
    def N(self):
        return self.coords.shape[0]

    @property
    def n_inst(self):
        return len(self.node_off) - 1

    def node_ionic(self):
        """[N, 6] per-node copy of the per-instance ionic parameters."""
        counts = np.diff(self.node_off)
        return np.repeat(self.ionic, counts, axis=0)


def _single(name, dim, coords, elems, tensor, sigma, **kw):
    N = coords.shape[0]
    return Problem(name=name, dim=dim, coords=coords, elems=elems.astype(np.int32),
                   elem_tensor=tensor, node_sigma=sigma,
                   node_off=np.array([0, N], dtype=np.int64),
                   elem_off=np.array([0, elems.shape[0]], dtype=np.int64),
                   ionic=np.array([AP_PARAMS]), v_init=np.zeros(N), w_init=np.zeros(N), **kw)


def config0(n=256, theta=0.0, n_steps=500):
    coords, elems = meshes.line_mesh(n, 1.0)
    tensor = np.full((elems.shape[0], 1, 1), 1e-3)
    stim = np.nonzero(coords[:, 0] <= 0.05)[0].astype(np.int32)
    return _single("1d-monodomain", 1, coords, elems, tensor, np.ones(n),
                   M=3, K=4, dt=0.1, n_steps=n_steps, theta=theta, stimuli=[(0.0, stim, 1.0)])


def config1(n=512, seed=1, theta=1e-7, n_steps=1000, K=4, width=16.0):
    coords, elems = meshes.square_tri_mesh(n, n, 2.0, 2.0)
    rng = np.random.default_rng(seed)
    phi = meshes.fiber_angles_2d(rng, n - 1, n - 1, width)
    tensor = np.repeat(meshes.rotated_tensor_2d(phi.ravel(), 1.2e-3, 3e-4), 2, axis=0)
    stim = np.nonzero(coords[:, 0] <= 0.1 + 1e-12)[0].astype(np.int32)
    return _single("2d-monodomain", 2, coords, elems, tensor, np.ones(coords.shape[0]),
                   M=4, K=K, dt=0.2, n_steps=n_steps, theta=theta, stimuli=[(0.0, stim, 1.0)])


def config2(n=128, seed=2, theta=1e-7, n_steps=1600, side=1.5, radius=0.1):
    coords, elems = meshes.cube_tet_mesh(n, side)
    zc = coords[elems, 2].mean(axis=1)
    phi = np.deg2rad(-60.0 + 120.0 * zc / side)
    fdir = np.stack([np.cos(phi), np.sin(phi), np.zeros_like(phi)], axis=1)
    tensor = meshes.fiber_tensor_3d(fdir, 1.2e-3, 3e-4)
    rng = np.random.default_rng(seed)
    lo, hi = 0.1 * side, 0.9 * side
    stimuli = []
    for t_on in (0.0, 120.0):
        c = rng.uniform(lo, hi, size=3)
        nodes = np.nonzero(np.sum((coords - c) ** 2, axis=1) <= radius ** 2)[0].astype(np.int32)
        stimuli.append((t_on, nodes, 1.0))
    return _single("3d-monodomain", 3, coords, elems, tensor, np.ones(coords.shape[0]),
                   M=4, K=4, dt=0.25, n_steps=n_steps, theta=theta, stimuli=stimuli)


def config4(n_inst=48, sizes=(96, 384), seed=4, theta=1e-7, n_steps=100, width=16.0,
            log_amp=0.3, target=False, target_seed=5, target_amp=0.1):
    """Batched instances; with target=True the conductivity of the target run
    is multiplied by exp(target_amp * g') with g' drawn from target_seed."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(sizes[0], sizes[1] + 1, size=n_inst)
    trng = np.random.default_rng(target_seed)
    coords_l, elems_l, sig_l, stim_l = [], [], [], []
    node_off, elem_off = [0], [0]
    for n in ns:
        c, e = meshes.square_tri_mesh(int(n), int(n), 2.0, 2.0)
        g = meshes.smoothed_gaussian(rng, (int(n), int(n)), width).ravel()
        sig = 1e-3 * np.exp(log_amp * g)
        if target:
            sig = sig * np.exp(target_amp * meshes.smoothed_gaussian(trng, (int(n), int(n)), width).ravel())
        base = node_off[-1]
        coords_l.append(c)
        elems_l.append(e + base)
        sig_l.append(sig)
        stim_l.append(base + np.nonzero(c[:, 0] <= 0.1 + 1e-12)[0])
        node_off.append(base + c.shape[0])
        elem_off.append(elem_off[-1] + e.shape[0])
    coords = np.concatenate(coords_l)
    elems = np.concatenate(elems_l).astype(np.int32)
    N = coords.shape[0]
    tensor = np.broadcast_to(np.eye(2), (elems.shape[0], 2, 2)).copy()
    return Problem(name="2d-batched", dim=2, coords=coords, elems=elems, elem_tensor=tensor,
                   node_sigma=np.concatenate(sig_l), node_off=np.array(node_off, dtype=np.int64),
                   elem_off=np.array(elem_off, dtype=np.int64),
                   ionic=np.tile(np.array(AP_PARAMS), (n_inst, 1)), M=3, K=4, dt=0.2,
                   n_steps=n_steps, theta=theta,
                   stimuli=[(0.0, np.concatenate(stim_l).astype(np.int32), 1.0)],
                   v_init=np.zeros(N), w_init=np.zeros(N))


def make(i, **kw):
    return {0: config0, 1: config1, 2: config2, 4: config4}[i](**kw)
