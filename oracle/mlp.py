"""Plain FP64 CPU reference of the band-column surrogate network.

TEST INFRASTRUCTURE ONLY, like the rest of this package: only ``tests/``,
``__graft_entry__.smoke()`` and ``bench.py``'s CPU baseline use it.  It shares
no code with the HIP path.

What the network computes.  For a source charge state k of a gas, a field
strength E_L and a step dt, the exact step of the rate chain (Eqs. (2)-(5),
Sec. 2) moves the population of level k to levels k, k+1, k+2, ...; the
first three entries of that column of exp(dt A) and the remainder (lumped at
k+3, where the locally reduced window of Sec. 3 puts it anyway) form a
probability vector of length 4.  The surrogate predicts it:

    u  = (log10 E_L - c_E) / s_E            (E range mapped to [-1, 1])
    v  = (log10 (dt omega_a) - c_t) / s_t   (dt / tau_a, tau_a = 1/omega_a)
    z1 = W1u u + W1v v + W1e emb[k] + b1          (64)
    h1 = relu(z1),  h2 = relu(W2 h1 + b2),  h3 = relu(W3 h2 + b3)   (64 each)
    z4 = W4 h3 + b4                                (4 logits)
    Q  = softmax(z4)

Weights are stored [out][in].  With ``bf16=True`` the arrays that feed the
matrix products of layers 2-4 (W2, W3, W4 and h1, h2, h3) are rounded to
bfloat16 (8 significant bits, round to nearest even) first, which is the
arithmetic of the device network; the backward pass then treats the rounding
as the identity (straight-through).  With ``bf16=False`` the network is a
smooth function of its parameters and the gradient is pinned by finite
differences.

Loss: cross entropy of the target column P against Q, averaged over the
batch, L = -(1/n) sum_s sum_j P_sj log Q_sj; dL/dz4 = (Q - P)/n.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

HIDDEN = 64
EMB = 16
BAND = 4

#: parameter blocks in storage order: name -> shape (Z substituted at run time)
_BLOCKS = (
    ("emb", ("Z", EMB)),
    ("W1u", (HIDDEN,)),
    ("W1v", (HIDDEN,)),
    ("W1e", (HIDDEN, EMB)),
    ("b1", (HIDDEN,)),
    ("W2", (HIDDEN, HIDDEN)),
    ("b2", (HIDDEN,)),
    ("W3", (HIDDEN, HIDDEN)),
    ("b3", (HIDDEN,)),
    ("W4", (BAND, HIDDEN)),
    ("b4", (BAND,)),
)


def block_shapes(Z: int):
    return [(name, tuple(Z if d == "Z" else d for d in shape)) for name, shape in _BLOCKS]


def nparams(Z: int) -> int:
    return sum(int(np.prod(s)) for _, s in block_shapes(Z))


def unpack(flat: np.ndarray, Z: int) -> dict:
    """Split the flat parameter vector into named FP64 arrays (views)."""
    flat = np.asarray(flat, dtype=np.float64)
    assert flat.size == nparams(Z)
    out, o = {}, 0
    for name, shape in block_shapes(Z):
        m = int(np.prod(shape))
        out[name] = flat[o:o + m].reshape(shape)
        o += m
    return out


def pack(blocks: dict, Z: int) -> np.ndarray:
    return np.concatenate([np.asarray(blocks[name], np.float64).ravel() for name, _ in block_shapes(Z)])


def bf16(x):
    """Round to the nearest bfloat16 value (8 significant bits, ties to even),
    returned as float64.  The exponent range of the inputs here never reaches
    bfloat16's subnormals or overflow."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)  # x = m 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.rint(m * 256.0) / 256.0, e)


@dataclass(frozen=True)
class Range:
    """Trained input range: field [GV/m] and step [s], and omega_a [1/s]."""
    E_lo: float = 10.0
    E_hi: float = 5000.0
    dt_lo: float = 0.02e-15
    dt_hi: float = 0.2e-15
    omega_a: float = 4.13e16

    def features(self, E, dt):
        lE0, lE1 = math.log10(self.E_lo), math.log10(self.E_hi)
        lt0, lt1 = math.log10(self.dt_lo * self.omega_a), math.log10(self.dt_hi * self.omega_a)
        u = (np.log10(np.abs(np.asarray(E, np.float64))) - 0.5 * (lE0 + lE1)) / (0.5 * (lE1 - lE0))
        v = (np.log10(np.asarray(dt, np.float64) * self.omega_a) - 0.5 * (lt0 + lt1)) / (0.5 * (lt1 - lt0))
        return u, np.broadcast_to(v, np.shape(u)).astype(np.float64)


def forward(params: np.ndarray, Z: int, u, v, k, bf16_ops: bool = True):
    """Network output for samples (u, v, k); returns (Q, cache)."""
    p = unpack(params, Z)
    rnd = bf16 if bf16_ops else (lambda a: np.asarray(a, np.float64))
    u = np.asarray(u, np.float64)
    v = np.asarray(v, np.float64)
    k = np.asarray(k, np.int64)
    z1 = np.outer(u, p["W1u"]) + np.outer(v, p["W1v"]) + p["emb"][k] @ p["W1e"].T + p["b1"]
    h1 = rnd(np.maximum(z1, 0.0))
    W2, W3, W4 = rnd(p["W2"]), rnd(p["W3"]), rnd(p["W4"])
    h2 = rnd(np.maximum(h1 @ W2.T + p["b2"], 0.0))
    h3 = rnd(np.maximum(h2 @ W3.T + p["b3"], 0.0))
    z4 = h3 @ W4.T + p["b4"]
    zm = z4 - z4.max(axis=1, keepdims=True)
    ez = np.exp(zm)
    Q = ez / ez.sum(axis=1, keepdims=True)
    cache = dict(p=p, u=u, v=v, k=k, h1=h1, h2=h2, h3=h3, W2=W2, W3=W3, W4=W4, Q=Q, zm=zm, ez=ez)
    return Q, cache


def layer_maps(params: np.ndarray, Z: int, u, v, k, z1, z2, z3):
    """The network one layer at a time, for checking an evaluation whose
    rounding decisions are given: z1, z2, z3 [n][64] are pre-activations of
    layers 1-3 as another evaluation computed them (before the rounding to
    bfloat16).  Returns the FP64 pre-activations each layer makes from the
    previous layer's given ones, rounded as the network rounds them:
        z1 = W1u u + W1v v + W1e emb[k] + b1,
        z2 = bf16(W2) bf16(relu(z1_given)) + b2,   likewise z3 from z2_given,
        z4 = bf16(W4) bf16(relu(z3_given)) + b4,
    each with the sum of the magnitudes of its terms (S1..S4), which bounds
    the rounding of any float32 summation order of those terms."""
    p = unpack(params, Z)
    u = np.asarray(u, np.float64)
    v = np.asarray(v, np.float64)
    k = np.asarray(k, np.int64)
    tu, tv = np.outer(u, p["W1u"]), np.outer(v, p["W1v"])
    out = {"z1": tu + tv + p["emb"][k] @ p["W1e"].T + p["b1"],
           "S1": np.abs(tu) + np.abs(tv) + np.abs(p["emb"][k]) @ np.abs(p["W1e"]).T + np.abs(p["b1"])}
    for i, (zg, Wn, bn) in enumerate(((z1, "W2", "b2"), (z2, "W3", "b3"), (z3, "W4", "b4")), start=2):
        h = bf16(np.maximum(np.asarray(zg, np.float64), 0.0))
        W = bf16(p[Wn])
        out[f"z{i}"] = h @ W.T + p[bn]
        out[f"S{i}"] = h @ np.abs(W).T + np.abs(p[bn])
    return out


def loss(Q, P):
    """Mean cross entropy; terms with P = 0 contribute nothing."""
    P = np.asarray(P, np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        t = np.where(P > 0, P * np.log(np.where(P > 0, Q, 1.0)), 0.0)
    return float(-t.sum() / P.shape[0])


def loss_and_grad(params: np.ndarray, Z: int, u, v, k, P, bf16_ops: bool = True, acts=None):
    """Loss and its gradient with respect to the flat parameter vector.
    acts = (h1, h2, h3) (optional): bfloat16 activations to take instead of
    the forward pass's own (the rounding decisions of another evaluation of
    the same network); the rest of the pass is unchanged."""
    Q, c = forward(params, Z, u, v, k, bf16_ops)
    if acts is not None:
        h1, h2, h3 = (np.asarray(a, np.float64) for a in acts)
        z4 = h3 @ c["W4"].T + c["p"]["b4"]
        zm = z4 - z4.max(axis=1, keepdims=True)
        Q = np.exp(zm) / np.exp(zm).sum(axis=1, keepdims=True)
        c.update(h1=h1, h2=h2, h3=h3, Q=Q)
    P = np.asarray(P, np.float64)
    n = P.shape[0]
    p = c["p"]
    g = {name: np.zeros(shape) for name, shape in block_shapes(Z)}
    dz4 = (Q - P) / n
    g["W4"] = dz4.T @ c["h3"]
    g["b4"] = dz4.sum(axis=0)
    dz3 = (dz4 @ c["W4"]) * (c["h3"] > 0)
    g["W3"] = dz3.T @ c["h2"]
    g["b3"] = dz3.sum(axis=0)
    dz2 = (dz3 @ c["W3"]) * (c["h2"] > 0)
    g["W2"] = dz2.T @ c["h1"]
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ c["W2"]) * (c["h1"] > 0)
    g["W1u"] = dz1.T @ c["u"]
    g["W1v"] = dz1.T @ c["v"]
    g["W1e"] = dz1.T @ p["emb"][c["k"]]
    g["b1"] = dz1.sum(axis=0)
    np.add.at(g["emb"], c["k"], dz1 @ p["W1e"])
    return loss(Q, P), pack(g, Z)


def adam_step(params, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015, Algorithm 1) with bias correction;
    t is the 1-based step count.  Returns new (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def band_update(N, lo, w, Z, cols, use):
    """Apply predicted band columns to windowed populations.

    N[w+1][n] holds levels lo..lo+w; cols[w][4][n] holds, for source slot s,
    the probabilities of landing at s, s+1, s+2 and s+3 or beyond.  The
    window top is t = min(w, Z - lo): destinations past it are lumped into
    it (it absorbs in the reduced system of Sec. 3), slot t keeps its own
    population, and slots past level Z stay empty.  Cells with use[c] false
    are returned unchanged."""
    N = np.asarray(N, np.float64)
    out = N.copy()
    n = N.shape[1]
    for c in range(n):
        if not use[c]:
            continue
        top = min(w, Z - int(lo[c]))
        if top <= 0:
            continue
        o = np.zeros(w + 1)
        o[top] = N[top, c]
        for s in range(top):
            for d in range(BAND):
                o[min(s + d, top)] += cols[s][d][c] * N[s, c]
        out[:, c] = o
    return out


def window_shift(N, lo, Z, eps):
    """Window shift at the start of a step (Sec. 3): while the lowest window
    level holds less than eps and is not the bare nucleus, fold it into the
    next level and move the window up by one."""
    N = np.array(N, np.float64)
    p = np.array(lo, np.int64)
    w = N.shape[0] - 1
    for c in range(N.shape[1]):
        while p[c] < Z and N[0, c] < eps:
            N[0, c] += N[1, c]
            N[1:w, c] = N[2:w + 1, c]
            N[w, c] = 0.0
            p[c] += 1
    return N, p


#: a source level whose rate gives W dt below this keeps its population
#: (identity column) in the surrogate form of the step
NEGLIGIBLE_XDT = 1e-9


def surrogate_step(orc, spec, Z, params, rng: Range, E, dt, pops, lo, w, eps, bf16_ops=True, cols_given=None,
                   negligible=None):
    """Reference of the surrogate form of the step: cells whose |E| lies in
    the trained range (and a step dt in range) take band columns after the
    window shift, the network's for source levels with W dt >= NEGLIGIBLE_XDT
    and the identity column for the others; all other cells take the exact
    step of the analytic oracle `orc.ionize_step`.  Also returns the window
    rates times dt, x[w][n] (0 past level Z-1).
    cols_given [w][4][n] (optional): network columns of another evaluation of
    the same network (its own bfloat16 rounding decisions) to use instead of
    this module's; negligible [w][n] (optional, bool): the identity decision
    per source slot instead of W dt < NEGLIGIBLE_XDT."""
    E = np.abs(np.asarray(E, np.float64))
    ana, alo = orc.ionize_step(spec, E, dt, np.asarray(pops, np.float64), np.asarray(lo, np.uint8), w, eps)
    dt_ok = rng.dt_lo <= dt <= rng.dt_hi
    use = (E >= rng.E_lo) & (E <= rng.E_hi) & dt_ok
    N, p = window_shift(pops, lo, Z, eps)
    use &= p < Z
    u, v = rng.features(np.where(use, E, rng.E_lo), dt)
    Wall = orc.rates(spec, np.where(np.isfinite(E), E, 0.0))
    x = np.zeros((w, E.size))
    cols = []
    for s in range(w):
        k = p + s
        ok = k < Z
        x[s, ok] = Wall[k[ok], np.nonzero(ok)[0]] * dt
        if cols_given is not None:
            Q = np.array(cols_given[s], np.float64)
        else:
            Q, _ = forward(params, Z, u, v, np.minimum(k, Z - 1), bf16_ops)
            Q = Q.T
        negl = x[s] < NEGLIGIBLE_XDT if negligible is None else np.asarray(negligible[s], bool)
        Q[:, negl] = np.array([1.0, 0.0, 0.0, 0.0])[:, None]
        cols.append(Q)
    band = band_update(N, p, w, Z, cols, use)
    out = np.where(use[None, :], band, ana)
    return out, np.where(use, p, alo).astype(np.uint8), use, x


def exact_band_columns(orc, spec, Z, E, dt, k):
    """Exact band columns (T[k..k+2, k] of exp(dt A) and the rest) from the
    analytic oracle: a unit population at level k stepped with a window of
    three rates and no shift.  dt may be a scalar or per sample."""
    E = np.asarray(E, np.float64)
    k = np.asarray(k, np.int64)
    dt = np.broadcast_to(np.asarray(dt, np.float64), E.shape)
    cols = np.zeros((BAND, E.size))
    for d in np.unique(dt):
        idx = np.nonzero(dt == d)[0]
        N = np.zeros((BAND, idx.size))
        N[0] = 1.0
        out, _ = orc.ionize_step(spec, E[idx], float(d), N, k[idx].astype(np.uint8), BAND - 1, 0.0)
        cols[:, idx] = out
    return cols
