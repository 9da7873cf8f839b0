"""Binary64 reference of the learned initial partition's network — TEST INFRASTRUCTURE.

The project proposes the initial k-way assignment of the coarsest graph (the
slot of §III-B's recursive bisection) with a small message-passing network.
This module writes that network in matrix form, in binary64, together with its
training loss and the loss gradient by hand-derived backpropagation:

    X      = [ c/c_max, deg/max_deg, Y_8 ],  Y_0 = seeded +-1 probes,
             Y_{t+1} = (Y_t + D^-1 A Y_t) / 2            (rows without neighbours: Y_{t+1} = Y_t)
    H_l    = ReLU(1 b_l^T + H_{l-1} Ws_l^T + M_l Wn_l^T),   M_l = D^-1 A H_{l-1}   (l = 1, 2, 3)
    Z      = 1 bh^T + H_3 Wh^T,   S = softmax(Z) row by row
    loss   = (1/Omega) sum_{(v,u) directed edges} w(v,u) BCE(p_vu, [t_v == t_u]),  p_vu = <S_v, S_u>
           + lam * k * sum_c (Q_c - 1/k)^2,   Q_c = sum_v c(v) S_v[c] / c(V)

A is the weighted adjacency matrix, D its row sums, Omega = sum of all entries
of A, t a target partition. p is clipped to [1e-6, 1 - 1e-6] (zero gradient
outside). The weights passed in are used as given (the GPU rounds its master
weights to bfloat16 first; tests pass that rounded copy here).

The binary32 inference that must match the GPU bit for bit is oracle/mpnn.c;
this module pins it (agreement within binary32 error) and is itself pinned by
central finite differences of its loss.
"""
import numpy as np
import scipy.sparse as sp

NPROBE, NWALK, NFEAT, HID = 16, 8, 18, 64
P_CLIP = 1e-6
_M64 = (1 << 64) - 1


def param_count(k):
    return (2 * HID * NFEAT + HID) + 2 * (2 * HID * HID + HID) + HID * k + k


def unpack(w, k):
    """Flat parameters -> list of (Ws, Wn, b) per layer and (Wh, bh)."""
    w = np.asarray(w, dtype=np.float64)
    assert w.size == param_count(k)
    layers, o = [], 0
    for din in (NFEAT, HID, HID):
        Ws = w[o:o + HID * din].reshape(HID, din); o += HID * din
        Wn = w[o:o + HID * din].reshape(HID, din); o += HID * din
        b = w[o:o + HID]; o += HID
        layers.append((Ws, Wn, b))
    Wh = w[o:o + HID * k].reshape(k, HID); o += HID * k
    bh = w[o:o + k]
    return layers, (Wh, bh)


def pack(layer_grads, head_grads):
    parts = []
    for gs, gn, gb in layer_grads:
        parts += [gs.ravel(), gn.ravel(), gb.ravel()]
    parts += [head_grads[0].ravel(), head_grads[1].ravel()]
    return np.concatenate(parts)


def _splitmix(x):
    z = (x + 0x9E3779B97F4A7C15) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def probes(n, seed):
    """Y_0[v][j] = -1 if the top bit of splitmix(splitmix(seed) ^ (16 v + j)) is set, else +1."""
    base = _splitmix(seed & _M64)
    Y = np.empty((n, NPROBE))
    for v in range(n):
        for j in range(NPROBE):
            Y[v, j] = -1.0 if _splitmix(base ^ (v * NPROBE + j)) >> 63 else 1.0
    return Y


def adjacency(g):
    n = len(g["xadj"]) - 1
    xadj = np.asarray(g["xadj"], dtype=np.int64)
    rows = np.repeat(np.arange(n), np.diff(xadj))
    w = np.ones(len(g["adjncy"])) if g.get("adjwgt") is None else np.asarray(g["adjwgt"], np.float64)
    return sp.csr_matrix((w, (rows, np.asarray(g["adjncy"], np.int64))), shape=(n, n))


def features(g, seed):
    n = len(g["xadj"]) - 1
    A = adjacency(g)
    wdeg = np.asarray(A.sum(axis=1)).ravel()
    has = wdeg > 0
    dinv = np.where(has, 1.0 / np.where(has, wdeg, 1.0), 0.0)
    Y = probes(n, seed)
    for _ in range(NWALK):
        Y = np.where(has[:, None], 0.5 * (Y + dinv[:, None] * (A @ Y)), Y)
    c = np.ones(n) if g.get("vwgt") is None else np.asarray(g["vwgt"], np.float64)
    deg = np.diff(np.asarray(g["xadj"], np.int64)).astype(np.float64)
    dmax = deg.max() if n else 0.0
    X = np.empty((n, NFEAT))
    X[:, 0] = c / c.max() if n else 0.0
    X[:, 1] = deg / dmax if dmax > 0 else 0.0
    X[:, 2:] = Y
    return X


def forward(g, k, w, seed=0, X=None):
    """Returns a cache dict with X, per-layer (H_in, M, H_out), logits Z."""
    layers, (Wh, bh) = unpack(w, k)
    A = adjacency(g)
    wdeg = np.asarray(A.sum(axis=1)).ravel()
    dinv = np.where(wdeg > 0, 1.0 / np.where(wdeg > 0, wdeg, 1.0), 0.0)
    H = features(g, seed) if X is None else np.asarray(X, np.float64)
    cache = {"A": A, "dinv": dinv, "X": H, "layers": []}
    for Ws, Wn, b in layers:
        M = dinv[:, None] * (A @ H)
        Hn = np.maximum(b[None, :] + H @ Ws.T + M @ Wn.T, 0.0)
        cache["layers"].append((H, M, Hn))
        H = Hn
    cache["Z"] = bh[None, :] + H @ Wh.T
    return cache


def _softmax(Z):
    e = np.exp(Z - Z.max(axis=1, keepdims=True))
    return e / e.sum(axis=1, keepdims=True)


def loss_and_grad(g, k, w, target, seed=0, lam=1.0, X=None):
    """(edge loss, balance loss, gradient w.r.t. the flat parameters)."""
    layers, (Wh, bh) = unpack(w, k)
    cache = forward(g, k, w, seed, X)
    A, dinv = cache["A"], cache["dinv"]
    n = A.shape[0]
    S = _softmax(cache["Z"])
    t = np.asarray(target)
    Ac = A.tocoo()
    omega = Ac.data.sum()
    p_raw = np.einsum("ij,ij->i", S[Ac.row], S[Ac.col])
    p = np.clip(p_raw, P_CLIP, 1.0 - P_CLIP)
    y = (t[Ac.row] == t[Ac.col]).astype(np.float64)
    edge_loss = -(Ac.data * (y * np.log(p) + (1 - y) * np.log(1 - p))).sum() / omega
    inside = (p_raw > P_CLIP) & (p_raw < 1.0 - P_CLIP)
    dldp = np.where(inside, -(y / p - (1 - y) / (1 - p)), 0.0) * Ac.data / omega
    # each directed term (v,u) feeds S_v (times S_u) and S_u (times S_v)
    G = sp.csr_matrix((dldp, (Ac.row, Ac.col)), shape=(n, n))
    gS = G @ S + G.T @ S
    c = np.ones(n) if g.get("vwgt") is None else np.asarray(g["vwgt"], np.float64)
    C = c.sum()
    Q = (c[:, None] * S).sum(axis=0) / C
    bal_loss = lam * k * ((Q - 1.0 / k) ** 2).sum()
    gS += (2.0 * lam * k * (Q - 1.0 / k))[None, :] * (c[:, None] / C)
    dZ = S * (gS - (S * gS).sum(axis=1, keepdims=True))
    H3 = cache["layers"][-1][2]
    gWh = dZ.T @ H3
    gbh = dZ.sum(axis=0)
    dH = dZ @ Wh
    lgrads = []
    for (Ws, Wn, b), (Hin, M, Hout) in zip(reversed(layers), reversed(cache["layers"])):
        dpre = dH * (Hout > 0)
        lgrads.append((dpre.T @ Hin, dpre.T @ M, dpre.sum(axis=0)))
        dM = dpre @ Wn
        dH = dpre @ Ws + A.T @ (dinv[:, None] * dM)
    lgrads.reverse()
    return edge_loss, bal_loss, pack(lgrads, (gWh, gbh))


def loss(g, k, w, target, seed=0, lam=1.0, X=None):
    e, b, _ = loss_and_grad(g, k, w, target, seed, lam, X)
    return e + b

