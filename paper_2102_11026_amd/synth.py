"""Seeded synthetic problem generator shared by the FP64 oracle and the HIP path.

This module only draws random numbers and lays out mesh / network data.  It
holds none of the method's arithmetic: no rest-shape matrices, masses,
derivatives, forces or solves (each side computes those itself).

Random numbers come from one counter-based generator, SplitMix64 (Steele,
Lea and Flood, "Fast splittable pseudorandom number generators", OOPSLA
2014), turned into 53-bit uniforms and then into normals by the Box-Muller
transform.  Every named sub-stream (``dec/3``, ``q0/0`` ...) gets its own
64-bit key, so adding a stream never shifts another one.

Workloads follow the paper's setting (Sec. 3.6 system, Sec. 6 experiments):
tet-meshed solids, a decoder MLP ``q -> u``, a cubature subset of elements
with weights that may come from a small weight-prediction MLP (Sec. 5.2),
implicit Euler with a fixed number of Newton iterations per step.  The
paper's meshes and trained networks are not available; regular grids split
into 5 tets and Xavier-initialised networks stand in for them.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

MASTER_SEED = 2102
_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


# --------------------------------------------------------------------------
# counter-based generator
# --------------------------------------------------------------------------
def _fnv1a64(text: str) -> np.uint64:
    h = 0xCBF29CE484222325
    for b in text.encode():
        h ^= b
        h = (h * 0x100000001B3) & 0xFFFFFFFFFFFFFFFF
    return np.uint64(h)


def _mix(z: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def stream_key(name: str, seed: int = MASTER_SEED) -> np.uint64:
    """64-bit key of a named sub-stream."""
    with np.errstate(over="ignore"):
        return _mix(np.array([np.uint64(seed) ^ _fnv1a64(name)], dtype=np.uint64))[0]


def raw64(name: str, count: int, seed: int = MASTER_SEED) -> np.ndarray:
    """SplitMix64 outputs 1..count of stream ``name`` (counter form)."""
    key = stream_key(name, seed)
    ctr = np.arange(1, count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix(key + ctr * _GAMMA)


def uniform(name: str, count: int, seed: int = MASTER_SEED) -> np.ndarray:
    """Uniforms in (0, 1]: top 53 bits of each draw, plus one ulp."""
    r = raw64(name, count, seed)
    return ((r >> np.uint64(11)).astype(np.float64) + 1.0) * (1.0 / 9007199254740992.0)


def normal(name: str, count: int, seed: int = MASTER_SEED) -> np.ndarray:
    """Standard normals by Box-Muller on consecutive uniform pairs."""
    pairs = (count + 1) // 2
    u = uniform(name, 2 * pairs, seed)
    u1, u2 = u[0::2], u[1::2]
    rad = np.sqrt(-2.0 * np.log(u1))
    z = np.empty(2 * pairs)
    z[0::2] = rad * np.cos(2.0 * np.pi * u2)
    z[1::2] = rad * np.sin(2.0 * np.pi * u2)
    return z[:count]


def permutation(name: str, n: int, seed: int = MASTER_SEED) -> np.ndarray:
    """Uniform random permutation of range(n) (argsort of 64-bit draws)."""
    return np.argsort(raw64(name, n, seed), kind="stable")


# --------------------------------------------------------------------------
# meshes
# --------------------------------------------------------------------------
# 5-tet split of a unit cube.  Corners are named by (dx, dy, dz) bits.  The
# "even" split keeps corner 000 with its three neighbours; the "odd" one is
# its mirror, so the face diagonals of neighbouring cubes agree.
_EVEN = [(0b000, 0b001, 0b010, 0b100), (0b011, 0b010, 0b001, 0b111),
         (0b101, 0b001, 0b100, 0b111), (0b110, 0b100, 0b010, 0b111),
         (0b001, 0b010, 0b100, 0b111)]
_ODD = [(0b001, 0b000, 0b011, 0b101), (0b010, 0b000, 0b011, 0b110),
        (0b100, 0b000, 0b101, 0b110), (0b111, 0b011, 0b101, 0b110),
        (0b000, 0b011, 0b101, 0b110)]


def grid_mesh(nx: int, ny: int, nz: int, spacing: float = 0.1):
    """Regular vertex grid split into 5 tets per cube.

    Vertex (i, j, k) sits at (i, j, k) * spacing with index i + nx*(j + ny*k).
    Returns (X (n,3) float64, tets (m,4) int32) with every tet positively
    oriented (vertex order swapped where needed).
    """
    ii, jj, kk = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    idx = lambda i, j, k: i + nx * (j + ny * k)
    n = nx * ny * nz
    X = np.zeros((n, 3))
    X[idx(ii, jj, kk).ravel(), 0] = ii.ravel() * spacing
    X[idx(ii, jj, kk).ravel(), 1] = jj.ravel() * spacing
    X[idx(ii, jj, kk).ravel(), 2] = kk.ravel() * spacing
    # cubes in k, j, i loop order (i fastest)
    ck, cj, ci = (a.ravel() for a in np.meshgrid(np.arange(nz - 1), np.arange(ny - 1), np.arange(nx - 1),
                                                 indexing="ij"))
    even = ((ci + cj + ck) % 2 == 0)[:, None, None]
    pat = np.where(even, np.asarray(_EVEN)[None], np.asarray(_ODD)[None])  # (cubes, 5, 4)
    tets = idx(ci[:, None, None] + (pat & 1), cj[:, None, None] + ((pat >> 1) & 1),
               ck[:, None, None] + ((pat >> 2) & 1)).reshape(-1, 4).astype(np.int32)
    # orientation: signed volume of the corner offsets
    e = X[tets[:, 1:]] - X[tets[:, :1]]
    s = np.einsum("ij,ij->i", e[:, 0], np.cross(e[:, 1], e[:, 2]))
    neg = s < 0
    tets[neg, 1], tets[neg, 2] = tets[neg, 2].copy(), tets[neg, 1].copy()
    return X, tets


# --------------------------------------------------------------------------
# problem bundle
# --------------------------------------------------------------------------
@dataclass
class Problem:
    """One simulated object.  All arrays float64 / int32, host memory."""
    name: str
    X: np.ndarray              # (n, 3) rest positions [m]
    tets: np.ndarray           # (m, 4) vertex ids, positive orientation
    pinned: np.ndarray         # (n,) uint8, 1 = Dirichlet vertex
    E: float
    nu: float
    rho: float
    gravity: np.ndarray        # (3,)
    dt: float
    U: np.ndarray              # (N, n_p) orthonormal, zero rows at pinned DOFs
    weights: List[np.ndarray]  # decoder W_l, (out, in)
    biases: List[np.ndarray]   # decoder b_l, (out,)
    act: str                   # hidden activation: tanh | elu | sin | identity
    cub_ids: np.ndarray        # (|C|,) tet ids
    cub_w: Optional[np.ndarray]            # fixed weights, or None -> W-net
    wnet_weights: Optional[List[np.ndarray]] = None
    wnet_biases: Optional[List[np.ndarray]] = None
    wnet_scale: float = 1.0
    r0: np.ndarray = None      # (R,) initial generalized coordinate [p; q]
    rdot0: np.ndarray = None   # (R,)
    steps: int = 1
    newton_iters: int = 1
    out_rows: int = 0          # rows of the output layer (>= N; prefix used)
    meta: dict = field(default_factory=dict)
    formulation: str = "full"  # "full" | "trimmed" (fictitious force dropped)
    fd_h: float = 0.0          # > 0: derivatives by central differences of this step

    @property
    def n(self) -> int:
        return self.X.shape[0]

    @property
    def N(self) -> int:
        return 3 * self.X.shape[0]

    @property
    def n_p(self) -> int:
        return self.U.shape[1]

    @property
    def n_q(self) -> int:
        return self.weights[0].shape[1]

    @property
    def R(self) -> int:
        return self.n_p + self.n_q

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


def xavier_mlp(widths, stream: str, seed: int = MASTER_SEED):
    """Xavier-normal weights (gain 1, std sqrt(2/(fan_in+fan_out))), zero biases."""
    Ws, bs = [], []
    for l in range(len(widths) - 1):
        fi, fo = widths[l], widths[l + 1]
        std = np.sqrt(2.0 / (fi + fo))
        Ws.append(normal(f"{stream}/{l}", fo * fi, seed).reshape(fo, fi) * std)
        bs.append(np.zeros(fo))
    return Ws, bs


def random_orthonormal(N: int, n_p: int, pinned_dof: np.ndarray, stream: str,
                       seed: int = MASTER_SEED) -> np.ndarray:
    """Orthonormal N x n_p basis supported on the free DOFs (QR of a Gaussian)."""
    if n_p == 0:
        return np.zeros((N, 0))
    free = np.flatnonzero(pinned_dof == 0)
    G = normal(stream, free.size * n_p, seed).reshape(free.size, n_p)
    Q, _ = np.linalg.qr(G)
    U = np.zeros((N, n_p))
    U[free] = Q
    return U


def _pins_k0(n: int, nx: int, ny: int) -> np.ndarray:
    p = np.zeros(n, dtype=np.uint8)
    p[: nx * ny] = 1  # vertices with k == 0
    return p


MATERIAL = dict(E=1.0e5, nu=0.45, rho=1000.0)
GRAVITY = np.array([0.0, -9.81, 0.0])
DT = 1.0 / 60.0


def bar_problem(name: str, grid, widths, act: str, *, n_p: int = 0, n_cub: int = 0,
                wnet_hidden=(64, 64), steps: int = 1, newton_iters: int = 1,
                q_std: float = 0.1, out_scale: float = 1.0, seed: int = MASTER_SEED,
                stream_prefix: str = "", instance: int = 0) -> Problem:
    """A bar on a regular grid pinned at its k = 0 face.

    ``widths`` are the decoder widths from n_q to the output size (3n).
    ``n_cub == 0`` means full quadrature (every tet, weight 1); otherwise a
    uniform sample of ``n_cub`` tets with weights from a softplus W-net
    evaluated on r (scaled so each weight is m/|C| at zero pre-activation).
    """
    nx, ny, nz = grid
    X, tets = grid_mesh(nx, ny, nz)
    n = X.shape[0]
    N = 3 * n
    assert widths[-1] >= N, "decoder output must cover every DOF"
    pinned = _pins_k0(n, nx, ny)
    pin_dof = np.repeat(pinned, 3)
    sp = stream_prefix
    Ws, bs = xavier_mlp(widths, sp + "dec", seed)
    Ws[-1] = Ws[-1] * out_scale
    U = random_orthonormal(N, n_p, pin_dof, f"{sp}U/{instance}", seed)
    n_q = widths[0]
    R = n_p + n_q
    m = tets.shape[0]
    if n_cub == 0:
        cub_ids = np.arange(m, dtype=np.int32)
        cub_w = np.ones(m)
        wW = wb = None
        wscale = 1.0
    else:
        cub_ids = np.sort(permutation(sp + "cub", m, seed)[:n_cub]).astype(np.int32)
        cub_w = None
        wW, wb = xavier_mlp([R, *wnet_hidden, n_cub], sp + "wnet", seed)
        wscale = (m / n_cub) / np.log(2.0)
    r0 = np.zeros(R)
    r0[n_p:] = q_std * normal(f"{sp}q0/{instance}", n_q, seed)
    return Problem(name=name, X=X, tets=tets, pinned=pinned, gravity=GRAVITY.copy(), dt=DT,
                   U=U, weights=Ws, biases=bs, act=act, cub_ids=cub_ids, cub_w=cub_w,
                   wnet_weights=wW, wnet_biases=wb, wnet_scale=wscale, r0=r0,
                   rdot0=np.zeros(R), steps=steps, newton_iters=newton_iters,
                   out_rows=widths[-1], meta=dict(grid=tuple(grid), widths=list(widths)),
                   **MATERIAL)


# Workload recipes ----------------------------------------------------------
C2_WIDTHS = [15, 64, 128, 256, 512, 512, 512, 512, 512, 256, 30000]


def config_plain_fp64() -> Problem:
    """192-vertex bar, r = 3, tanh decoder [3,32,64,128,576], full quadrature,
    20 steps x 3 Newton iterations."""
    return bar_problem("bar192_r3", (4, 4, 12), [3, 32, 64, 128, 576], "tanh",
                       steps=20, newton_iters=3)


def config_single_10k(instance: int = 0) -> Problem:
    """10,000-vertex bar (20x20x25, 43,320 tets), r = 15, 10-layer ELU decoder,
    500 cubature tets weighted by a 15->64->64->500 softplus W-net,
    100 steps x 4 Newton iterations."""
    return bar_problem("bar10k_r15", (20, 20, 25), C2_WIDTHS, "elu", n_cub=500,
                       steps=100, newton_iters=4, instance=instance)


SERVE_A_WIDTHS = [5, 64, 128, 256, 256, 128, 6000]
SERVE_C_WIDTHS = [30, 64, 128, 256, 512, 1024, 1024, 1024, 1024, 1024, 512, 256, 150000]


def config_serve_a(instance: int = 0) -> Problem:
    """Serving class A: 2,000-vertex bar (10 x 10 x 20), r = 5, depth-6 ELU
    decoder, full quadrature (7,695 tets), 120 steps x 4 iterations."""
    return bar_problem("serveA_2k_r5", (10, 10, 20), SERVE_A_WIDTHS, "elu", steps=120, newton_iters=4,
                       instance=instance, stream_prefix="serveA/")


def config_serve_b(instance: int = 0) -> Problem:
    """Serving class B: the 10,000-vertex, r = 15 problem, 120 steps."""
    return config_single_10k(instance).replace(steps=120)


def config_serve_c(instance: int = 0) -> Problem:
    """Serving class C: 50,000-vertex bar (20 x 20 x 125, 223,820 tets),
    r = 30, depth-12 ELU decoder with widths up to 1024, 6,600 cubature tets
    weighted by a 30 -> 64 -> 64 -> 6600 weight net, 120 steps x 4 iterations."""
    return bar_problem("serveC_50k_r30", (20, 20, 125), SERVE_C_WIDTHS, "elu", n_cub=6600, steps=120,
                       newton_iters=4, instance=instance, stream_prefix="serveC/")


def fibonacci_sphere(n: int) -> np.ndarray:
    """n nearly uniform unit vectors (golden-angle spiral)."""
    k = np.arange(n) + 0.5
    z = 1.0 - 2.0 * k / n
    rad = np.sqrt(1.0 - z * z)
    phi = np.pi * (3.0 - np.sqrt(5.0)) * k
    return np.stack([rad * np.cos(phi), rad * np.sin(phi), z], axis=1)


ROD_LENGTHS = (20, 30, 40, 60)
ROD_WIDTHS = [5, 32, 64, 128, 720]


ROD_OUT_SCALE = 0.25


def rod_decoder(seed: int = MASTER_SEED, out_scale: float = ROD_OUT_SCALE):
    """Shared rod decoder: tanh trunk 5 -> 32 -> 64 -> 128 and one 720 x 128
    head; a rod of length L uses the first 12 L output rows.  The head is
    scaled by out_scale: at 1 the random decoder inverts tets of most rods in
    their initial configuration (one element across the rod), at 1/4 every
    rod starts with det F > 0.35 and none inverts over its 60 steps."""
    Ws, bs = xavier_mlp(ROD_WIDTHS, "rods/dec", seed)
    Ws[-1] = Ws[-1] * out_scale
    return Ws, bs


def rod_problem(i: int, n_rods: int = 320, decoder=None, seed: int = MASTER_SEED) -> Problem:
    """Rod i of a puffer-ball-like set: a 2 x 2 x L vertex grid (L drawn from
    {20, 30, 40, 60}) along the i-th direction of a Fibonacci sphere, its root
    face centred at 0.5 m on that direction and pinned; n_p = 10 linear basis
    of its own, n_q = 5 shared tanh decoder, full quadrature."""
    L = int(np.asarray(ROD_LENGTHS)[raw64("rods/len", n_rods, seed)[i] % np.uint64(len(ROD_LENGTHS))])
    X0, tets = grid_mesh(2, 2, L)
    d = fibonacci_sphere(n_rods)[i]
    ref = np.array([0.0, 0.0, 1.0]) if abs(d[2]) < 0.9 else np.array([1.0, 0.0, 0.0])
    e1 = ref - d * (ref @ d)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(d, e1)
    # local (x, y, z) = (across 1, across 2, along the rod), right-handed frame
    X = 0.5 * d + (X0[:, 0:1] - 0.05) * e1 + (X0[:, 1:2] - 0.05) * e2 + X0[:, 2:3] * d
    n = X.shape[0]
    N = 3 * n
    pinned = np.zeros(n, dtype=np.uint8)
    pinned[:4] = 1
    Ws, bs = decoder if decoder is not None else rod_decoder(seed)
    U = random_orthonormal(N, 10, np.repeat(pinned, 3), f"rods/U/{i}", seed)
    R = 10 + 5
    r0 = np.zeros(R)
    r0[10:] = 0.1 * normal(f"rods/q0/{i}", 5, seed)
    m = tets.shape[0]
    return Problem(name=f"rod{i}_L{L}", X=X, tets=tets, pinned=pinned, gravity=GRAVITY.copy(), dt=DT, U=U,
                   weights=Ws, biases=bs, act="tanh", cub_ids=np.arange(m, dtype=np.int32), cub_w=np.ones(m),
                   r0=r0, rdot0=np.zeros(R), steps=60, newton_iters=3, out_rows=ROD_WIDTHS[-1],
                   meta=dict(L=L, rod=i), **MATERIAL)


def config_rods(n_rods: int = 320):
    """All rods of the batched workload, sharing one decoder."""
    dec = rod_decoder()
    return [rod_problem(i, n_rods, dec) for i in range(n_rods)]


def lsd_problem() -> Problem:
    """Fast-motion problem of the fictitious-force comparison: a soft 3 x 3 x 10
    vertex bar (E = 1e3), n_p = 0, full quadrature, a sine decoder
    [3, 32, 32, 32, 270] whose first layer has 10x the Xavier gain (the
    latent map is curved over one step's displacement), output scaled by
    0.05, started at rest shape with an abrupt latent velocity of 2 N(0, 1)."""
    p = tiny_problem(grid=(3, 3, 10), widths=(3, 32, 32, 32, 270), act="sin", n_p=0, name="lsd", q_std=0.0,
                     out_scale=0.05)
    W = [w.copy() for w in p.weights]
    W[0] = W[0] * 10.0
    return p.replace(E=1e3, weights=W, rdot0=2.0 * normal("lsd/rdot0", p.R), steps=15, newton_iters=6)


def tiny_problem(grid=(2, 2, 3), widths=(2, 4, 4, 36), act="tanh", n_p=0, n_cub=0,
                 q_std=0.1, name="tiny", instance=0, out_scale=1.0) -> Problem:
    return bar_problem(name, grid, list(widths), act, n_p=n_p, n_cub=n_cub, q_std=q_std,
                       instance=instance, out_scale=out_scale, stream_prefix=name + "/")


# --------------------------------------------------------------------------
# coupled multi-domain scenes (the puffer ball / cactus setting of Sec. 6.8)
# --------------------------------------------------------------------------
@dataclass
class CoupledScene:
    """A core domain and rods tied to it: ties[k] (4, 2) pairs (vertex of rod
    k, vertex of the core) whose copies are joined by springs of stiffness
    kappa [N/m]."""
    core: Problem
    rods: List[Problem]
    ties: List[np.ndarray]
    kappa: float
    steps: int = 1
    newton_iters: int = 1


# outward normal and in-face axes (e1 x e2 = n) of the five free faces of a
# grid pinned at k = 0: top, +x, -x, +y, -y
_FACES = (
    ("top", (0, 0, 1), (1, 0, 0), (0, 1, 0)),
    ("+x", (1, 0, 0), (0, 1, 0), (0, 0, 1)),
    ("-x", (-1, 0, 0), (0, 0, 1), (0, 1, 0)),
    ("+y", (0, 1, 0), (0, 0, 1), (1, 0, 0)),
    ("-y", (0, -1, 0), (1, 0, 0), (0, 0, 1)),
)


def attach_sites(grid):
    """Unit squares of the five free faces of a grid pinned at k = 0 at which
    a rod can be rooted, no two sharing a vertex (odd offsets, away from the
    face edges and from the pinned face): list of (corner (i, j, k), n, e1, e2)."""
    nx, ny, nz = grid
    size = np.array([nx, ny, nz])
    out = []
    for name, n, e1, e2 in _FACES:
        n, e1, e2 = (np.array(v) for v in (n, e1, e2))
        base = np.where(n > 0, size - 1, 0) * np.abs(n)
        a1, a2 = int(np.flatnonzero(e1)[0]), int(np.flatnonzero(e2)[0])
        for s1 in range(1, size[a1] - 2, 2):
            for s2 in range(1, size[a2] - 2, 2):
                corner = base + s1 * e1 + s2 * e2
                out.append((tuple(int(c) for c in corner), n, e1, e2))
    return out


def rod_frame_basis(X: np.ndarray, n_p: int, stream: str, seed: int = MASTER_SEED) -> np.ndarray:
    """(3n, n_p) orthonormal basis of a free rod: its three translations and
    three infinitesimal rotations about the centre of its root face (the first
    four vertices), then Gaussian directions, orthonormalised by QR, so that
    the linear subspace can follow the motion of what the rod is tied to."""
    n = X.shape[0]
    c = X[:4].mean(axis=0)
    cols = []
    for a in range(3):
        t = np.zeros((n, 3))
        t[:, a] = 1.0
        cols.append(t.ravel())
    for a in range(3):
        ax = np.zeros(3)
        ax[a] = 1.0
        cols.append(np.cross(ax, X - c).ravel())
    extra = max(n_p - 6, 0)
    G = normal(stream, 3 * n * extra, seed).reshape(3 * n, extra)
    M = np.column_stack(cols[: min(6, n_p)] + [G])
    Q, _ = np.linalg.qr(M)
    return Q[:, :n_p]


def coupled_scene(name: str, core_grid, n_rods: int, rod_lengths, *, core_np: int, core_widths, rod_np: int,
                  rod_widths, act: str = "tanh", kappa: float = 1.0e5, core_out_scale: float = 0.25,
                  rod_out_scale: float = 0.25, q_std: float = 0.02, steps: int = 1, newton_iters: int = 3,
                  seed: int = MASTER_SEED) -> CoupledScene:
    """A core (a grid pinned at its k = 0 face, n_p linear plus a decoder of
    its own, full quadrature) with n_rods 2 x 2 x L rods rooted on unit squares
    of its five free faces (chosen by a seeded permutation of the sites), each
    rod's root face a copy of the square's four core vertices tied to them by
    springs.  Rods share one decoder (rod_widths[-1] >= 12 max L, a rod using
    the first 12 L rows) and have their own frame basis (rod_frame_basis);
    nothing of a rod is pinned.  Full quadrature everywhere; initial latent
    q ~ N(0, q_std^2), linear coordinates and velocities zero."""
    sp = name + "/"
    nx, ny, nz = core_grid
    Xc, tc = grid_mesh(nx, ny, nz)
    nc = Xc.shape[0]
    pin_c = _pins_k0(nc, nx, ny)
    Wc, bc = xavier_mlp(core_widths, sp + "core/dec", seed)
    Wc[-1] = Wc[-1] * core_out_scale
    assert core_widths[-1] >= 3 * nc
    Uc = random_orthonormal(3 * nc, core_np, np.repeat(pin_c, 3), sp + "core/U", seed)
    nqc = core_widths[0]
    rc0 = np.zeros(core_np + nqc)
    rc0[core_np:] = q_std * normal(sp + "core/q0", nqc, seed)
    mc = tc.shape[0]
    core = Problem(name=sp + "core", X=Xc, tets=tc, pinned=pin_c, gravity=GRAVITY.copy(), dt=DT, U=Uc,
                   weights=Wc, biases=bc, act=act, cub_ids=np.arange(mc, dtype=np.int32), cub_w=np.ones(mc),
                   r0=rc0, rdot0=np.zeros(core_np + nqc), steps=steps, newton_iters=newton_iters,
                   out_rows=core_widths[-1], meta=dict(grid=tuple(core_grid), widths=list(core_widths)), **MATERIAL)
    sites = attach_sites(core_grid)
    assert n_rods <= len(sites), (n_rods, len(sites))
    pick = np.sort(permutation(sp + "sites", len(sites), seed)[:n_rods])
    Ws, bs = xavier_mlp(rod_widths, sp + "rods/dec", seed)
    Ws[-1] = Ws[-1] * rod_out_scale
    Ls = np.asarray(rod_lengths)[raw64(sp + "rods/len", n_rods, seed) % np.uint64(len(rod_lengths))]
    cidx = lambda v: int(v[0] + nx * (v[1] + ny * v[2]))
    rods, ties = [], []
    nqr = rod_widths[0]
    for k, s in enumerate(pick):
        corner, n, e1, e2 = sites[int(s)]
        L = int(Ls[k])
        X0, tr = grid_mesh(2, 2, L)
        assert rod_widths[-1] >= X0.size
        P0 = Xc[cidx(corner)]
        X = P0 + X0[:, 0:1] * e1 + X0[:, 1:2] * e2 + X0[:, 2:3] * n
        nv = X.shape[0]
        U = rod_frame_basis(X, rod_np, sp + f"rods/U/{k}", seed)
        r0 = np.zeros(rod_np + nqr)
        r0[rod_np:] = q_std * normal(sp + f"rods/q0/{k}", nqr, seed)
        m = tr.shape[0]
        rods.append(Problem(name=sp + f"rod{k}_L{L}", X=X, tets=tr, pinned=np.zeros(nv, np.uint8),
                            gravity=GRAVITY.copy(), dt=DT, U=U, weights=Ws, biases=bs, act=act,
                            cub_ids=np.arange(m, dtype=np.int32), cub_w=np.ones(m), r0=r0,
                            rdot0=np.zeros(rod_np + nqr), steps=steps, newton_iters=newton_iters,
                            out_rows=rod_widths[-1], meta=dict(L=L, site=int(s)), **MATERIAL))
        root = [(a, b) for b in (0, 1) for a in (0, 1)]     # rod vertices 0..3 = (a, b, 0)
        ties.append(np.array([[a + 2 * b, cidx(np.array(corner) + a * e1 + b * e2)] for a, b in root],
                             dtype=np.int64))
    return CoupledScene(core=core, rods=rods, ties=ties, kappa=kappa, steps=steps, newton_iters=newton_iters)


def config_coupled_tiny(n_rods: int = 2) -> CoupledScene:
    """Small coupled scene for the parity tests: a 4 x 4 x 5 core (n_p = 4,
    tanh decoder [3, 16, 16, 240]) with rods of 3 or 4 vertex layers (n_p = 6,
    shared decoder [3, 16, 16, 48])."""
    return coupled_scene("coupled_tiny", (4, 4, 5), n_rods, (3, 4), core_np=4, core_widths=[3, 16, 16, 240],
                         rod_np=6, rod_widths=[3, 16, 16, 48], q_std=0.05, steps=4, newton_iters=3)


def config_puffer(n_rods: int = 320) -> CoupledScene:
    """Puffer-ball-like coupled scene: a 21 x 21 x 21 core (9,261 vertices,
    40,000 tets) pinned at one face, n_p = 10 plus an n_q = 6 tanh decoder
    [6, 32, 64, 128, 27783], and 320 rods of 2 x 2 x L vertices (L from
    {20, 30, 40, 60}) rooted on its five free faces, each with n_p = 10 and the
    shared n_q = 5 decoder [5, 32, 64, 128, 720]; full quadrature, tie springs
    of 1e5 N/m, 60 steps x 3 Newton iterations."""
    return coupled_scene("puffer", (21, 21, 21), n_rods, ROD_LENGTHS, core_np=10,
                         core_widths=[6, 32, 64, 128, 3 * 21 ** 3], rod_np=10, rod_widths=ROD_WIDTHS,
                         steps=60, newton_iters=3)


# --------------------------------------------------------------------------
# neural cubature training sets (Sec. 5)
# --------------------------------------------------------------------------
@dataclass
class CubatureTraining:
    """Poses and initial networks of one neural cubature training run.

    ``prob`` gives the mesh, material, U and decoder; ``poses`` (P x R) stand
    in for the simulated training poses of Sec. 5 (normal draws at the
    magnitudes the simulator visits).  The weight net has widths
    [R, *hidden, c_max] (Xavier, zero biases) with c_max = n_c0 + K *
    alternations rows in its last layer, one per element C will hold; scale =
    (m / c_max) / ln 2.  ``theta`` holds the selection net's 170 parameters in
    the order G0 (3 x 8), G1 (8 x 8), A1 (8 x 8), a1 (8), A2 (8), a2, c: the
    matrices Xavier-normal, the rest zero."""
    prob: Problem
    poses: np.ndarray
    wnet_weights: List[np.ndarray]
    wnet_biases: List[np.ndarray]
    scale: float
    theta: np.ndarray
    n_c0: int
    K: int
    alternations: int
    epochs: int
    lr: float = 1.0e-3

    @property
    def c_max(self) -> int:
        return self.n_c0 + self.K * self.alternations


def cubature_training(prob: Problem, n_poses: int, n_c0: int, K: int, alternations: int, epochs: int,
                      hidden=(64, 64), p_std: float = 0.02, q_std: float = 0.1, name: str = "cubtrain",
                      seed: int = MASTER_SEED) -> CubatureTraining:
    R, n_p = prob.R, prob.n_p
    z = normal(f"{name}/poses", n_poses * R, seed).reshape(n_poses, R)
    poses = np.concatenate([p_std * z[:, :n_p], q_std * z[:, n_p:]], axis=1)
    c_max = n_c0 + K * alternations
    Ws, bs = xavier_mlp([R, *hidden, c_max], f"{name}/wnet", seed)
    m = prob.tets.shape[0]
    scale = (m / c_max) / np.log(2.0)
    parts = []
    for k, (fi, fo) in enumerate([(3, 8), (8, 8), (8, 8)]):
        parts.append(normal(f"{name}/snet/{k}", fi * fo, seed) * np.sqrt(2.0 / (fi + fo)))
    parts.append(np.zeros(8))
    parts.append(normal(f"{name}/snet/3", 8, seed) * np.sqrt(2.0 / 9.0))
    parts.append(np.zeros(2))
    theta = np.concatenate(parts)
    return CubatureTraining(prob=prob, poses=poses, wnet_weights=Ws, wnet_biases=bs, scale=scale, theta=theta,
                            n_c0=n_c0, K=K, alternations=alternations, epochs=epochs)


def config_cubature_tiny() -> CubatureTraining:
    """Small training run for the parity tests: a 3 x 3 x 4 bar (36 vertices,
    60 tets), n_p = 2 plus a tanh decoder [3, 8, 8, 108] (output layer scaled
    by 0.05); 12 poses, C from 4
    samples plus 4 per alternation over 3 alternations of 4 epochs, weight net
    [5, 16, 16, 16]."""
    p = tiny_problem(grid=(3, 3, 4), widths=(3, 8, 8, 108), act="tanh", n_p=2, name="cubtiny", out_scale=0.05)
    return cubature_training(p, 12, 4, 4, 3, 4, hidden=(16, 16), q_std=0.3, name="cubtiny")


def config_cubature_bar10k(n_poses: int = 1024) -> CubatureTraining:
    """Training run on the 10,000-vertex bar (43,320 tets, r = 15, the ELU
    decoder of the headline problem): n_poses poses, C from 20 Voronoi samples
    plus 20 per alternation up to 500 elements, weight net 15 -> 64 -> 64 ->
    500, 15 epochs per net per alternation (Sec. 5)."""
    p = config_single_10k().replace(cub_ids=np.arange(43320, dtype=np.int32), cub_w=np.ones(43320),
                                   wnet_weights=None, wnet_biases=None, wnet_scale=1.0)
    return cubature_training(p, n_poses, 20, 20, 24, 15, name="cubbar10k")
