"""Neural cubature training in FP64 (test infrastructure only).

Sec. 5 trains two networks in alternation on a set of poses r_p:
- the weight net W maps a pose r to non-negative weights of the cubature
  elements C; it is the net the simulator evaluates once per step (Sec. 5.2).
  It has the run-time form of this library: an MLP with a softplus after
  every layer times a fixed scale (oracle/wnet.py).  Its last layer holds a
  row for each of the at most c_max elements C will ever hold, in the order
  they join C; only the first |C| rows are in use;
- the selection net S, a graph convolutional network on the mesh (Sec. 5.1,
  eq. of the graph convolution): two convolutions with 8 channels,
  h_i' = sin(sum_{j in N(i)} h_j Gamma / sqrt(d_i d_j)) over the one-ring
  N(i) (the vertex itself included, d_i = |N(i)|), applied to the vertex
  displacements; each element takes the mean of its four vertices' features;
  two fully connected layers (8 -> 8 with sin, 8 -> 1) give a logit z_e; a
  softmax over the elements outside C times e^c (c trained) gives the
  scores s_e.

Training data (Sec. 5.1): per pose the reduced force of every element,
Ft_e(r) = Jt_e(r)^T f_e(u(r)), and the full-quadrature reduced force
f(r) = sum_e Ft_e(r).  Losses (Sec. 5.2), relative squared norms averaged
over the P poses:
    L_W = (1/P) sum_p |f_p - sum_{j<|C|} w_j(r_p) Ft_{C_j},p|^2 / |f_p|^2
    L_S = (1/P) sum_p |fb_p - sum_{e not in C} s_e(u_p) Ft_e,p|^2 / |fb_p|^2
with fb_p = f_p - sum_j w_j(r_p) Ft_{C_j},p, the residual force left by the
current cubature (eq. of the residual force).

One alternation: `epochs` full-batch Adam steps (Kingma and Ba 2015) on W,
the residuals fb_p with the updated W, `epochs` Adam steps on S, then the K
elements outside C with the largest score averaged over the poses join C
(ties to the lower element id).  Each net keeps its Adam state across
alternations; a row of W's last layer that is not in use has zero gradient,
so Adam leaves it and its moments untouched until its element joins.

Farthest-point sampling of the element centroids (from element 0) gives the
initial Voronoi samples of Sec. 5.2.

Parity: the element forces sum to the gradient of the elastic energy along
the decoded subspace (central differences); both loss gradients against
central differences; Adam's first step in closed form; L_W = 0 when C holds
every element at weight one; the selection on a hand-made score table.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np

from . import fem
from .wnet import softplus

S_CH = 8                                 # channels of both graph convolutions
S_LAYOUT = [("G0", (3, S_CH)), ("G1", (S_CH, S_CH)), ("A1", (S_CH, S_CH)), ("a1", (S_CH,)),
            ("A2", (S_CH,)), ("a2", ()), ("c", ())]
S_SIZE = sum(int(np.prod(s)) for _, s in S_LAYOUT)   # 170


def sigmoid(x):
    return 0.5 * (1.0 + np.tanh(0.5 * x))


# ---------------------------------------------------------------------------
# training data (Sec. 5.1)
# ---------------------------------------------------------------------------
def pose_jacobian(inst, r):
    """u(r) (N,) and Jt(r) = [U, J] (N, R)."""
    p = inst.p
    n_p = inst.n_p
    z = np.zeros(inst.n_q)
    d = inst.decode(r[n_p:], z, z)
    u = (p.U @ r[:n_p] if n_p else 0.0) + d["m"]
    return u, np.concatenate([p.U, d["J"]], axis=1)


def element_forces(inst, r):
    """(F, f, u): F[e] = Jt_e^T f_e at pose r for every element (m, R), the
    full-quadrature reduced force f = sum_e F[e] and the displacement u."""
    p = inst.p
    u, Jt = pose_jacobian(inst, r)
    fe, _ = fem.element_force_stiffness(p.X, p.tets, u, inst.Bm, inst.Ve, inst.mu, inst.lam)
    F = np.einsum("eir,ei->er", Jt[fem.tet_dofs(p.tets)], fe)
    return F, F.sum(axis=0), u


# ---------------------------------------------------------------------------
# weight net: z_{l+1} = softplus(W_l z_l + b_l), w = scale z_L (first nC rows)
# ---------------------------------------------------------------------------
def wnet_forward(Ws, bs, scale, nC, r):
    L = len(Ws)
    zs, As = [np.asarray(r, np.float64)], []
    for l in range(L):
        W, b = (Ws[l][:nC], bs[l][:nC]) if l == L - 1 else (Ws[l], bs[l])
        a = W @ zs[-1] + b
        As.append(a)
        zs.append(softplus(a))
    return scale * zs[-1], (zs, As)


def loss_W(Ws, bs, scale, C, data):
    """L_W and its gradient (arrays shaped like Ws, bs).  data: [(r, F, f)]."""
    P, L, nC = len(data), len(Ws), len(C)
    loss = 0.0
    gW = [np.zeros_like(W) for W in Ws]
    gb = [np.zeros_like(b) for b in bs]
    for r, F, f in data:
        w, (zs, As) = wnet_forward(Ws, bs, scale, nC, r)
        FC = F[C]
        res = f - FC.T @ w
        nf = f @ f
        loss += (res @ res) / nf / P
        dz = scale * (-2.0 / (P * nf)) * (FC @ res)
        for l in range(L - 1, -1, -1):
            da = dz * sigmoid(As[l])
            gW[l][:da.size] += np.outer(da, zs[l])
            gb[l][:da.size] += da
            W = Ws[l][:nC] if l == L - 1 else Ws[l]
            dz = W.T @ da
    return loss, gW, gb


# ---------------------------------------------------------------------------
# selection net (Sec. 5.1)
# ---------------------------------------------------------------------------
def mesh_graph(tets, n):
    """Dense normalised adjacency of the one-ring graph, self included:
    A_ij = 1 / sqrt(d_i d_j) for j in N(i), d_i = |N(i)|."""
    adj = np.zeros((n, n), bool)
    for a in range(4):
        for b in range(4):
            adj[tets[:, a], tets[:, b]] = True
    d = adj.sum(axis=1).astype(np.float64)
    return adj / np.sqrt(np.outer(d, d))


def s_unpack(theta):
    out, o = {}, 0
    for name, shape in S_LAYOUT:
        k = int(np.prod(shape))
        out[name] = theta[o:o + k].reshape(shape) if shape else float(theta[o])
        o += k
    return out


def s_pack(parts):
    return np.concatenate([np.atleast_1d(np.asarray(parts[name], np.float64)).ravel() for name, _ in S_LAYOUT])


def snet_forward(theta, Ahat, tets, u, cand):
    """Logits z (m,) and scores s over the candidates cand."""
    t = s_unpack(theta)
    H0 = Ahat @ u.reshape(-1, 3)
    P1 = H0 @ t["G0"]
    H1 = Ahat @ np.sin(P1)
    P2 = H1 @ t["G1"]
    g = np.sin(P2)[tets].mean(axis=1)
    Q = g @ t["A1"].T + t["a1"]
    Y = np.sin(Q)
    z = Y @ t["A2"] + t["a2"]
    zc = z[cand]
    e = np.exp(zc - zc.max())
    pi = e / e.sum()
    s = np.exp(t["c"]) * pi
    return z, s, dict(H0=H0, P1=P1, H1=H1, P2=P2, g=g, Q=Q, Y=Y, pi=pi)


def snet_backward(theta, Ahat, tets, cand, cache, ds):
    """Gradient (flat) of a scalar with dL/ds = ds."""
    t = s_unpack(theta)
    pi = cache["pi"]
    s = np.exp(t["c"]) * pi
    gc = float(ds @ s)
    dz = np.zeros(tets.shape[0])
    dz[cand] = s * (ds - ds @ pi)
    gA2 = dz @ cache["Y"]
    ga2 = float(dz.sum())
    dQ = np.outer(dz, t["A2"]) * np.cos(cache["Q"])
    gA1 = dQ.T @ cache["g"]
    ga1 = dQ.sum(axis=0)
    dg = dQ @ t["A1"]
    dX2 = np.zeros((Ahat.shape[0], S_CH))
    for a in range(4):
        np.add.at(dX2, tets[:, a], dg / 4.0)
    dP2 = dX2 * np.cos(cache["P2"])
    gG1 = cache["H1"].T @ dP2
    dP1 = (Ahat.T @ (dP2 @ t["G1"].T)) * np.cos(cache["P1"])
    gG0 = cache["H0"].T @ dP1
    return s_pack(dict(G0=gG0, G1=gG1, A1=gA1, a1=ga1, A2=gA2, a2=ga2, c=gc))


def loss_S(theta, Ahat, tets, cand, data_s):
    """L_S and its gradient (flat).  data_s: [(u, F, fb)]."""
    P = len(data_s)
    loss, grad = 0.0, np.zeros(S_SIZE)
    for u, F, fb in data_s:
        _, s, cache = snet_forward(theta, Ahat, tets, u, cand)
        Fc = F[cand]
        res = fb - Fc.T @ s
        nf = fb @ fb
        loss += (res @ res) / nf / P
        grad += snet_backward(theta, Ahat, tets, cand, cache, -2.0 / (P * nf) * (Fc @ res))
    return loss, grad


def select_top(scores, cand, K):
    """The K candidates with the largest score, ties to the lower element id."""
    order = sorted(range(len(cand)), key=lambda i: (-scores[i], cand[i]))
    return [int(cand[i]) for i in order[:K]]


# ---------------------------------------------------------------------------
# Adam (Kingma and Ba 2015)
# ---------------------------------------------------------------------------
@dataclass
class Adam:
    lr: float = 1e-3
    b1: float = 0.9
    b2: float = 0.999
    eps: float = 1e-8
    m: List[np.ndarray] = field(default_factory=list)
    v: List[np.ndarray] = field(default_factory=list)
    t: int = 0

    def step(self, params, grads):
        """Updates the arrays in params in place."""
        if not self.m:
            self.m = [np.zeros_like(p) for p in params]
            self.v = [np.zeros_like(p) for p in params]
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        for p, g, m, v in zip(params, grads, self.m, self.v):
            m[...] = self.b1 * m + (1.0 - self.b1) * g
            v[...] = self.b2 * v + (1.0 - self.b2) * (g * g)
            p -= self.lr * (m / c1) / (np.sqrt(v / c2) + self.eps)


# ---------------------------------------------------------------------------
# the alternation
# ---------------------------------------------------------------------------
def voronoi_samples(X, tets, k):
    """k elements by farthest-point sampling of the centroids from element 0."""
    c = X[tets].mean(axis=1)
    pick = [0]
    d = np.linalg.norm(c - c[0], axis=1)
    for _ in range(k - 1):
        e = int(np.argmax(d))
        pick.append(e)
        d = np.minimum(d, np.linalg.norm(c - c[e], axis=1))
    return pick


@dataclass
class TrainResult:
    C: list
    Ws: list
    bs: list
    theta: np.ndarray
    loss_w: list          # per alternation, per epoch (before each Adam step)
    loss_s: list
    added: list           # per alternation, the K elements that joined C
    mean_scores: list     # per alternation, (candidates, averaged scores)


def train(inst, rs, Ws, bs, scale, theta, C0, K, alternations, epochs, lr=1e-3, data=None):
    """Alternating neural cubature training from the given initial nets
    (copied; the weight net's last layer has a row per element C may hold)."""
    p = inst.p
    m = p.tets.shape[0]
    if data is None:
        data = [element_forces(inst, r) for r in rs]
    Ahat = mesh_graph(p.tets, p.n)
    Ws = [W.copy() for W in Ws]
    bs = [b.copy() for b in bs]
    theta = np.array(theta, np.float64, copy=True)
    C = list(C0)
    adW, adS = Adam(lr=lr), Adam(lr=lr)
    res = TrainResult(C, Ws, bs, theta, [], [], [], [])
    for _ in range(alternations):
        dw = [(r, F, f) for r, (F, f, _) in zip(rs, data)]
        lw = []
        for _ in range(epochs):
            L, gW, gb = loss_W(Ws, bs, scale, C, dw)
            lw.append(L)
            adW.step(Ws + bs, gW + gb)
        inC = np.zeros(m, bool)
        inC[C] = True
        cand = np.flatnonzero(~inC)
        ds = []
        for r, (F, f, u) in zip(rs, data):
            w, _ = wnet_forward(Ws, bs, scale, len(C), r)
            ds.append((u, F, f - F[C].T @ w))
        ls = []
        for _ in range(epochs):
            L, g = loss_S(theta, Ahat, p.tets, cand, ds)
            ls.append(L)
            adS.step([theta], [g])
        mean = np.zeros(cand.size)
        for u, _, _ in ds:
            _, s, _ = snet_forward(theta, Ahat, p.tets, u, cand)
            mean += s / len(ds)
        add = select_top(mean, cand, K)
        C += add
        res.loss_w.append(lw)
        res.loss_s.append(ls)
        res.added.append(add)
        res.mean_scores.append((cand, mean))
    res.theta = theta
    return res
