"""Seeded problem generators (no KKT arithmetic lives here).

Conventions shared by every consumer:

* Spatial nodes of an ``n[0] x n[1] x n[2]``-element uniform hex mesh of the box
  ``[0,len0] x [0,len1] x [0,len2]`` are numbered ``g = i + (n0+1)*(j + (n1+1)*k)``
  (x fastest).  Elements are numbered the same way with ``n`` instead of ``n+1``.
* Time levels are ``t^m = m*T/M`` for ``m = 0..M``.
* ``data[m, s]`` is the noisy concentration at sensor ``s`` and level ``m``.
* Dirichlet faces are a bitmask: bit 0 = {x=0}, 1 = {x=len0}, 2 = {y=0},
  3 = {y=len1}, 4 = {z=0}, 5 = {z=len2}.  Every other face is Neumann.

Random draws use NumPy's PCG64 (``numpy.random.default_rng(seed)``) in a fixed
order: coefficient field, then sources, then noise.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

DTO = 0
OTD = 1
H1H1 = 0   # regularisation of eq. (3): time and space gradients of f
H1L2 = 1   # the H1-L2 regularisation of Example 2: time gradient and L2 norm of f


@dataclass
class Problem:
    """One inverse-source instance: everything that defines F_h and b."""
    n: tuple            # elements per axis (nx, ny, nz)
    M: int              # time steps; levels 0..M
    a_elem: np.ndarray  # float64[nz*ny*nx], x fastest
    v: tuple            # constant velocity (vx, vy, vz)
    beta1: float
    beta2: float
    sensor_node: np.ndarray   # int32[s], global spatial node ids
    data: np.ndarray          # float64[M+1, s]
    length: tuple = (1.0, 1.0, 1.0)
    T: float = 1.0
    dirichlet_faces: int = 0b000011
    variant: int = DTO
    reg: int = H1H1
    name: str = ""
    f_true: Optional[np.ndarray] = None   # float64[M+1, N] when kept (diagnostic)
    data_clean: Optional[np.ndarray] = None  # noise-free sensor values (for fresh noise draws)
    noise: float = 0.0

    @property
    def nodes(self):
        return tuple(k + 1 for k in self.n)

    @property
    def N(self):
        nx, ny, nz = self.nodes
        return nx * ny * nz

    @property
    def V(self):
        return self.N * (self.M + 1)

    @property
    def unknowns(self):
        return 3 * self.V


@dataclass
class SolverConfig:
    """Preconditioner and Krylov settings attached to a configuration."""
    parts: tuple = (2, 2, 2, 2)      # subdomains in x, y, z, t
    overlap: int = 1
    restart: int = 30
    rtol: float = 1e-6
    maxit: int = 10000
    flexible: bool = False
    precision: str = "f64"           # factor / coarse precision
    coarse_factor: Optional[tuple] = None   # (fx, fy, fz, ft) for two-level


# --------------------------------------------------------------------------
# building blocks
# --------------------------------------------------------------------------

def sensor_lattice(n: int, k: int) -> np.ndarray:
    """k interior node indices on an n-element axis: round-half-up of (i+1)n/(k+1)."""
    i = np.arange(k)
    return ((i + 1) * 2 * n + (k + 1)) // (2 * (k + 1))


def _node_coords(n, length):
    xs = [np.linspace(0.0, length[d], n[d] + 1) for d in range(3)]
    Z, Y, X = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
    return X.ravel(), Y.ravel(), Z.ravel()


def _smooth_field(rng, nterms=8):
    """Parameters of g(x) = sum_k c_k cos(2 pi m_k.x + phi_k)."""
    modes = []
    while len(modes) < nterms:
        m = rng.integers(0, 3, size=3)
        if m.any():
            modes.append(m)
    modes = np.array(modes, dtype=np.float64)
    c = rng.standard_normal(nterms)
    phi = rng.uniform(0.0, 2.0 * np.pi, nterms)
    return modes, c, phi


def _eval_field(params, X, Y, Z):
    modes, c, phi = params
    g = np.zeros_like(X)
    for k in range(len(c)):
        g += c[k] * np.cos(2 * np.pi * (modes[k, 0] * X + modes[k, 1] * Y + modes[k, 2] * Z) + phi[k])
    return g


class _Coefficient:
    """a(x) = exp(0.5 g(x)), g normalised so that max over mesh nodes |g| = 1."""

    def __init__(self, rng, n, length):
        self.params = _smooth_field(rng)
        X, Y, Z = _node_coords(n, length)
        gmax = np.abs(_eval_field(self.params, X, Y, Z)).max()
        self.scale = 1.0 / gmax if gmax > 0 else 1.0

    def __call__(self, X, Y, Z):
        return np.exp(0.5 * self.scale * _eval_field(self.params, X, Y, Z))


class _Sources:
    """f(x,t) = I(t) * sum_k A_k exp(-|x - c_k(t)|^2 / w^2), c_k linear in t."""

    def __init__(self, starts, ends, width, amp=1.0, sin_intensity=True):
        self.p = np.asarray(starts, dtype=np.float64).reshape(-1, 3)
        self.q = np.asarray(ends, dtype=np.float64).reshape(-1, 3)
        self.w = float(width)
        self.amp = float(amp)
        self.sin_intensity = sin_intensity

    def __call__(self, X, Y, Z, t):
        out = np.zeros_like(X)
        for k in range(self.p.shape[0]):
            c = self.p[k] + t * (self.q[k] - self.p[k])
            r2 = (X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2
            out += self.amp * np.exp(-r2 / self.w ** 2)
        if self.sin_intensity:
            out *= np.sin(np.pi * t)
        return out


def _dirichlet_nodes(n, faces):
    nx, ny, nz = (k + 1 for k in n)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    m = np.zeros(i.size, dtype=bool)
    for bit, (arr, val) in enumerate([(i, 0), (i, nx - 1), (j, 0), (j, ny - 1), (k, 0), (k, nz - 1)]):
        if faces >> bit & 1:
            m |= arr == val
    return m


def _forward_fv(n, length, M, T, coef, v, src, faces, sensor_node, substeps=2, refine=2):
    """Observation generator: the model of eq. (1) forward-solved on a finer mesh.

    Node-centred finite volumes on the mesh refined ``refine`` times per axis
    (every inversion node is a node of it), advanced by the Douglas
    alternating-direction scheme with ``refine * substeps`` steps per time
    step of the inversion (C implementation in ``fvgen.c``).  Diffusion uses
    dual cells with a(x) at edge midpoints, convection -v.grad C central
    differences inside and one-sided ones on boundary nodes; Dirichlet nodes
    hold C = 0.  A different discretisation on a finer mesh than the
    inversion's, as the paper produces its data (Section 4).  Returns C at the
    sensor nodes for t^m = m T / M, m = 0..M, with C(., 0) = 0.
    """
    import ctypes
    from . import clib
    r = int(refine)
    nn = [r * n[d] + 1 for d in range(3)]
    h = [length[d] / (r * n[d]) for d in range(3)]
    xs = [np.arange(nn[d]) * h[d] for d in range(3)]
    mids = [0.5 * (xs[d][:-1] + xs[d][1:]) for d in range(3)]
    amid = []
    for d in range(3):
        ax = [mids[e] if e == d else xs[e] for e in range(3)]
        Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
        a = coef(X.ravel(), Y.ravel(), Z.ravel()) if coef is not None else np.ones(X.size)
        amid.append(np.ascontiguousarray(a, dtype=np.float64))
    dmask = np.ascontiguousarray(_dirichlet_nodes(tuple(k - 1 for k in nn), faces).astype(np.uint8))
    NX, NY = n[0] + 1, n[1] + 1
    sn = np.asarray(sensor_node, dtype=np.int64)
    i, j, k = sn % NX, (sn // NX) % NY, sn // (NX * NY)
    sens = np.ascontiguousarray(r * i + nn[0] * (r * j + nn[1] * r * k), dtype=np.int32)
    out = np.zeros((M + 1, sens.size))
    nsteps = M * r * substeps
    P = ctypes.c_void_p
    arr = lambda a: a.ctypes.data_as(P)
    nn_c = np.array(nn, dtype=np.int32)
    h_c = np.array(h, dtype=np.float64)
    v_c = np.array(v, dtype=np.float64)
    p_c = np.ascontiguousarray(src.p, dtype=np.float64)
    q_c = np.ascontiguousarray(src.q, dtype=np.float64)
    rc = clib.lib().fv_forward(arr(nn_c), arr(h_c), float(T), int(nsteps), int(r * substeps), arr(amid[0]),
                               arr(amid[1]), arr(amid[2]), arr(v_c), arr(dmask), int(src.p.shape[0]), arr(p_c),
                               arr(q_c), float(src.w), float(src.amp), int(bool(src.sin_intensity)),
                               int(sens.size), arr(sens), arr(out))
    if rc != 0:
        raise RuntimeError("fv_forward failed")
    return out


# --------------------------------------------------------------------------
# configurations
# --------------------------------------------------------------------------

def _make(name, n, M, seed, *, smooth_coef, nsrc, width, sin_int, starts=None, ends=None,
          sensors=None, noise=0.01, beta=1e-4, v=(1.0, 0.5, 0.25), keep_f=False,
          length=(1.0, 1.0, 1.0), T=1.0, faces=0b000011, variant=DTO, reg=H1H1):
    rng = np.random.default_rng(seed)
    n = tuple(int(k) for k in n)
    coef = _Coefficient(rng, n, length) if smooth_coef else None
    if starts is None:
        starts = rng.uniform(0.2, 0.8, size=(nsrc, 3))
        ends = rng.uniform(0.2, 0.8, size=(nsrc, 3))
    src = _Sources(starts, ends, width, sin_intensity=sin_int)
    # element coefficients sampled at element centroids
    h = [length[d] / n[d] for d in range(3)]
    ez, ey, ex = np.meshgrid(*(np.arange(n[d]) + 0.5 for d in (2, 1, 0)), indexing="ij")
    cx, cy, cz = ex.ravel() * h[0], ey.ravel() * h[1], ez.ravel() * h[2]
    a_elem = coef(cx, cy, cz) if coef is not None else np.ones(cx.size)
    if sensors is None:
        raise ValueError("sensor set required")
    sensor_node = np.asarray(sensors, dtype=np.int32)
    clean = _forward_fv(n, length, M, T, coef, v, src, faces, sensor_node)
    u = rng.uniform(-1.0, 1.0, size=clean.shape)
    data = clean * (1.0 + noise * u)
    f_true = None
    if keep_f:
        X, Y, Z = _node_coords(n, length)
        f_true = np.stack([src(X, Y, Z, m * T / M) for m in range(M + 1)])
    return Problem(n=n, M=int(M), a_elem=np.ascontiguousarray(a_elem, dtype=np.float64), v=tuple(v),
                   beta1=float(beta), beta2=float(beta), sensor_node=sensor_node,
                   data=np.ascontiguousarray(data), length=tuple(length), T=float(T),
                   dirichlet_faces=faces, variant=variant, reg=reg, name=name, f_true=f_true,
                   data_clean=clean, noise=float(noise))


def redraw_noise(prob, seed):
    """New observations of the same concentrations: fresh multiplicative uniform noise."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(-1.0, 1.0, size=prob.data_clean.shape)
    return prob.data_clean * (1.0 + prob.noise * u)


def lattice_nodes(n, k):
    """Global ids of the k^3 lattice sensor nodes on an n^3-element mesh."""
    idx = sensor_lattice(n, k)
    nn = n + 1
    kk, jj, ii = np.meshgrid(idx, idx, idx, indexing="ij")
    return (ii + nn * (jj + nn * kk)).ravel().astype(np.int32)


CONFIGS = {
    # tiny plain FP64 configuration (about 37k unknowns)
    "cube8x16": dict(n=8, M=16, seed=0, smooth_coef=False, nsrc=1, width=0.1, sin_int=False,
                 starts=[[0.25, 0.25, 0.25]], ends=[[0.75, 0.75, 0.75]], lattice=3,
                 solver=SolverConfig(parts=(2, 2, 2, 2), overlap=1, restart=30)),
    # single-GPU FP64 configuration (7.0M unknowns)
    "cube32x64": dict(n=32, M=64, seed=1, smooth_coef=True, nsrc=2, width=0.08, sin_int=True, lattice=4,
                 solver=SolverConfig(parts=(4, 4, 4, 8), overlap=2, restart=50)),
    # two-level mixed precision configuration (34M unknowns), coarse 12^3 x 24
    "cube48x96": dict(n=48, M=96, seed=2, smooth_coef=True, nsrc=2, width=0.08, sin_int=True, lattice=5,
                 solver=SolverConfig(parts=(4, 4, 4, 8), overlap=1, restart=50, flexible=True,
                                     coarse_factor=(4, 4, 4, 4))),
}


def config(name):
    c = dict(CONFIGS[name])
    return c


def make_problem(name="cube8x16", *, seed=None, n=None, M=None, keep_f=False, variant=DTO, **over):
    """Build the seeded Problem of a named configuration (optionally resized)."""
    c = dict(CONFIGS[name])
    c.update(over)
    solver = c.pop("solver")
    lattice = c.pop("lattice")
    if seed is not None:
        c["seed"] = seed
    if n is not None:
        c["n"] = n
    if M is not None:
        c["M"] = M
    nn = c.pop("n")
    sensors = lattice_nodes(nn, lattice)
    prob = _make(name, (nn, nn, nn), c.pop("M"), c.pop("seed"), sensors=sensors,
                 keep_f=keep_f, variant=variant, **c)
    return prob, dataclasses.replace(solver)


def make_custom(n, M, seed, *, sensors=None, lattice=2, nsrc=1, width=0.15, smooth_coef=True,
                beta=1e-4, noise=0.01, v=(1.0, 0.5, 0.25), faces=0b000011, variant=DTO,
                length=(1.0, 1.0, 1.0), T=1.0, reg=H1H1):
    """Small instances of arbitrary (possibly anisotropic) shape for tests."""
    n = tuple(int(k) for k in n)
    if sensors is None:
        rng_s = np.random.default_rng(seed + 7919)
        nn = tuple(k + 1 for k in n)
        # distinct interior nodes (never on a face)
        cand = [(i, j, k) for k in range(1, n[2]) for j in range(1, n[1]) for i in range(1, n[0])]
        pick = rng_s.choice(len(cand), size=min(lattice ** 3, len(cand)), replace=False)
        sensors = np.array([cand[p][0] + nn[0] * (cand[p][1] + nn[1] * cand[p][2]) for p in sorted(pick)])
    return _make("custom", n, M, seed, smooth_coef=smooth_coef, nsrc=nsrc, width=width, sin_int=True,
                 sensors=sensors, noise=noise, beta=beta, v=v, faces=faces, variant=variant,
                 length=length, T=T, reg=reg)


BATCH_N = (8, 12, 16, 20, 24)
BATCH_M = (16, 24, 32, 48)


def _uneven_instance(i, seed, rng, n, M):
    """One instance of the uneven batch: 1-3 sources, 27-64 sensors, noise 0.5-2%,
    beta in {1e-5, 1e-4, 1e-3}, drawn from rng after the sizes."""
    nsrc = int(rng.integers(1, 4))
    s = int(rng.integers(27, 65))
    noise = float(rng.uniform(0.005, 0.02))
    beta = float(rng.choice([1e-5, 1e-4, 1e-3]))
    nn = n + 1
    interior = (n - 1) ** 3
    pick = np.sort(rng.choice(interior, size=s, replace=False))
    i1 = pick % (n - 1) + 1
    j1 = (pick // (n - 1)) % (n - 1) + 1
    k1 = pick // (n - 1) ** 2 + 1
    sensors = (i1 + nn * (j1 + nn * k1)).astype(np.int32)
    return _make(f"batch{i}", (n, n, n), M, seed + 10000, smooth_coef=True, nsrc=nsrc,
                 width=0.08, sin_int=True, sensors=sensors, noise=noise, beta=beta)


def batch_instances(count=64, base_seed=3000, max_n=None, max_M=None):
    """Uneven batch: n in {8..24}, M in {16..48}, 1-3 sources, 27-64 sensors.

    max_n / max_M clamp the drawn sizes (small stand-ins for tests); every
    other draw is unchanged."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(base_seed + i)
        n = int(rng.choice(BATCH_N))
        M = int(rng.choice(BATCH_M))
        if max_n is not None:
            n = min(n, int(max_n))
        if max_M is not None:
            M = min(M, int(max_M))
        out.append(_uneven_instance(i, base_seed + i, rng, n, M))
    return out


def class_instances(n, M, count=4, base_seed=9000):
    """Instances of one size class (n, M) of the uneven batch, the other draws as there."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(base_seed + 101 * n + 7 * M + i)
        rng.choice(BATCH_N), rng.choice(BATCH_M)   # keep the draw sequence of batch_instances
        out.append(_uneven_instance(i, base_seed + 101 * n + 7 * M + i, rng, n, M))
    return out


def manufactured_solution(prob, seed=0, terms=3):
    """A seeded smooth space-time vector in the unknown layout (level, node, slot):
    per slot a sum of `terms` separable products cos(2 pi (k.x) + phase) in
    x, y, z and t with integer wave numbers 0..2, the C and G slots multiplied
    by sin(pi x / len0) (zero on the x = 0 and x = len0 faces, the Dirichlet
    faces of the benchmark problems).  Used as the exact solution x* of a
    manufactured system F x* = b."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = prob.nodes
    axes = [np.linspace(0.0, prob.length[0], nx), np.linspace(0.0, prob.length[1], ny),
            np.linspace(0.0, prob.length[2], nz), np.linspace(0.0, prob.T, prob.M + 1)]
    lens = list(prob.length) + [prob.T]
    out = np.zeros((prob.M + 1, nz, ny, nx, 3))
    for c in range(3):
        acc = np.zeros((prob.M + 1, nz, ny, nx))
        for _ in range(terms):
            amp = rng.standard_normal()
            f = [np.cos(2 * np.pi * rng.integers(0, 3) * axes[d] / lens[d] + rng.uniform(0, 2 * np.pi))
                 for d in range(4)]
            acc += amp * f[3][:, None, None, None] * f[2][None, :, None, None] * f[1][None, None, :, None] \
                * f[0][None, None, None, :]
        if c < 2:
            acc *= np.sin(np.pi * axes[0] / lens[0])[None, None, None, :]
        out[..., c] = acc
    return out.ravel()
