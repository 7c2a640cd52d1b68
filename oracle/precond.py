"""Learned per-shell damping gains (oracle).

TEST INFRASTRUCTURE ONLY: see the package docstring.

The paper's damped step (Eq. dampstep) preconditions the residual with the
fixed operator x0 / (E0 + T_k).  The learned extension multiplies that
operator, for each state alpha and each of S = 8 equal-width shells of |k|
(up to the zone corner |k|max = sqrt(3) (n/2) 2 pi / L), by a gain
g = 4 sigmoid(o) predicted by a small MLP.  This module writes out, plainly
and in FP64:

* the shells, the residual's spectral power per shell and the features;
* the MLP (4 -> 128 -> 128 -> 128 -> 1, ReLU) evaluated with its weights
  rounded to bfloat16 (round to nearest even), the weighted mean-square loss
  of the gains and its gradient by backpropagation;
* the training targets: the gains that minimise, to first order in the step
  and with the mean field frozen, the residual after the step,
  |r - sum_s g_s (h - <h>) d_s|^2 with d_s the plain damped residual
  restricted to shell s (real g_s, ridge 1e-6 tr(G)/S, clamped to [0, 4]).

Parameter layout (flat float array): W1[128][4], b1[128], W2[128][128], b2,
W3[128][128], b3, W4[128], b4.  Sample rows: [x0, x1, x2, x3, target, weight].
"""
from __future__ import annotations

import math
from typing import Dict, Tuple

import numpy as np
import scipy.fft as sfft

from .grid import _WORKERS, Grid
from .physics import MeanField, apply_h

S = 8          # |k| shells
PIN = 4        # features
PH = 128       # hidden width
GMAX = 4.0     # largest gain
NPAR = PH * PIN + PH + 2 * (PH * PH + PH) + PH + 1


def bf16_round(x: np.ndarray) -> np.ndarray:
    """float32 values rounded to bfloat16 (nearest, ties to even), as float64."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = u + 0x7FFF + ((u >> 16) & 1)
    u = (u & 0xFFFF0000).astype(np.uint32)
    return u.view(np.float32).astype(np.float64)


def unpack(P: np.ndarray) -> Dict[str, np.ndarray]:
    """Split the flat parameter vector into the layer matrices and biases."""
    P = np.asarray(P, dtype=np.float64)
    sizes = [("W1", (PH, PIN)), ("b1", (PH,)), ("W2", (PH, PH)), ("b2", (PH,)),
             ("W3", (PH, PH)), ("b3", (PH,)), ("W4", (PH,)), ("b4", ())]
    out, off = {}, 0
    for name, shape in sizes:
        cnt = int(np.prod(shape)) if shape else 1
        out[name] = P[off:off + cnt].reshape(shape) if shape else P[off]
        off += cnt
    assert off == NPAR
    return out


def pack(p: Dict[str, np.ndarray]) -> np.ndarray:
    return np.concatenate([np.ravel(p[k]) for k in
                           ("W1", "b1", "W2", "b2", "W3", "b3", "W4")] + [[p["b4"]]])


def forward(Pr: np.ndarray, X: np.ndarray):
    """MLP output o and the hidden activations, for parameters Pr used as given."""
    p = unpack(Pr)
    x = np.asarray(X, dtype=np.float64)[:, :PIN]
    a1 = x @ p["W1"].T + p["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(a2, 0.0)
    a3 = h2 @ p["W3"].T + p["b3"]
    h3 = np.maximum(a3, 0.0)
    o = h3 @ p["W4"] + p["b4"]
    return o, (x, a1, h1, a2, h2, a3, h3)


def gains_of(o: np.ndarray) -> np.ndarray:
    return GMAX / (1.0 + np.exp(-o))


def loss(Pr: np.ndarray, rows: np.ndarray) -> float:
    """sum_b w_b (g_b - t_b)^2 / sum_b w_b for parameters Pr used as given."""
    o, _ = forward(Pr, rows)
    t, w = rows[:, 4].astype(np.float64), rows[:, 5].astype(np.float64)
    return float(np.sum(w * (gains_of(o) - t) ** 2) / np.sum(w))


def loss_and_grad(P: np.ndarray, rows: np.ndarray) -> Tuple[float, np.ndarray]:
    """Loss at the bfloat16-rounded parameters and its gradient with respect to
    them (the gradient the FP32 master copy is updated with), by the chain rule
    through the layers in reverse order."""
    Pr = bf16_round(P)
    p = unpack(Pr)
    o, (x, a1, h1, a2, h2, a3, h3) = forward(Pr, rows)
    t, w = rows[:, 4].astype(np.float64), rows[:, 5].astype(np.float64)
    wsum = np.sum(w)
    sg = 1.0 / (1.0 + np.exp(-o))
    g = GMAX * sg
    L = float(np.sum(w * (g - t) ** 2) / wsum)
    do = 2.0 * w * (g - t) / wsum * GMAX * sg * (1.0 - sg)
    d3 = np.outer(do, p["W4"]) * (a3 > 0)
    d2 = (d3 @ p["W3"]) * (a2 > 0)
    d1 = (d2 @ p["W2"]) * (a1 > 0)
    grad = {"W4": h3.T @ do, "b4": do.sum(),
            "W3": d3.T @ h2, "b3": d3.sum(axis=0),
            "W2": d2.T @ h1, "b2": d2.sum(axis=0),
            "W1": d1.T @ x, "b1": d1.sum(axis=0)}
    return L, pack(grad)


def adam(P, G, M, V, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015, bias-corrected moments)."""
    M = b1 * M + (1 - b1) * G
    V = b2 * V + (1 - b2) * G * G
    Pn = P - lr * (M / (1 - b1 ** step)) / (np.sqrt(V / (1 - b2 ** step)) + eps)
    return Pn, M, V


# ------------------------------------------------------------------ shells

def mode_indices(n: int) -> np.ndarray:
    """Signed FFT mode numbers 0..n/2-1, -n/2..-1."""
    return np.fft.fftfreq(n, d=1.0 / n).round().astype(np.int64)


def shell_of_modes(n: int) -> np.ndarray:
    """Shell of every grid mode [z, y, x]: s = floor(S |k| / |k|max), capped at
    S - 1, with |k| = kunit sqrt(m2) and |k|max = kunit sqrt(3) n / 2, decided
    exactly as the count of j in 1..S-1 with 4 S^2 m2 >= 3 j^2 n^2."""
    m = mode_indices(n)
    m2 = m[:, None, None] ** 2 + m[None, :, None] ** 2 + m[None, None, :] ** 2
    s = np.zeros(m2.shape, dtype=np.int64)
    for j in range(1, S):
        s += (3 * j * j * n * n <= 4 * S * S * m2)
    return s


def shell_power(r: np.ndarray, g: Grid) -> np.ndarray:
    """P[alpha, s] = sum over modes of shell s and both spin components of
    |F r_alpha(k)|^2 (unnormalised transform; only ratios are used)."""
    fk = sfft.fftn(r, axes=(-3, -2, -1), workers=_WORKERS)
    pw = (np.abs(fk) ** 2).sum(axis=1)                  # [state][z][y][x]
    sh = shell_of_modes(g.n)
    return np.stack([pw[:, sh == s].sum(axis=1) for s in range(S)], axis=1)


def features(pow_: np.ndarray, eps: np.ndarray, e0: float, hb2m: float, g: Grid
             ) -> np.ndarray:
    """Rows [alpha*S + s] = [x0, x1, x2, x3, 0, w]:
    x0 = shell centre |k| / |k|max, x1 = <h>_alpha / E0,
    x2 = log10(share of the residual power in s + 1e-12) / 6 + 1,
    x3 = T at the shell centre / E0, w = share of the residual power in s."""
    kmax = math.sqrt(3.0) * (g.n // 2) * 2.0 * math.pi / g.L
    tot = pow_.sum(axis=1, keepdims=True)
    frac = np.where(tot > 0, pow_ / np.where(tot > 0, tot, 1.0), 0.0)
    m = pow_.shape[0]
    rows = np.zeros((m * S, 6))
    kc = (np.arange(S) + 0.5) / S
    for a in range(m):
        rows[a * S:(a + 1) * S, 0] = kc
        rows[a * S:(a + 1) * S, 1] = eps[a] / e0
        rows[a * S:(a + 1) * S, 2] = np.log10(frac[a] + 1e-12) / 6.0 + 1.0
        rows[a * S:(a + 1) * S, 3] = hb2m * (kc * kmax) ** 2 / e0
        rows[a * S:(a + 1) * S, 5] = frac[a]
    return rows


def gained_damping(r: np.ndarray, gain: np.ndarray, g: Grid, hb2m: float, x0: float,
                   e0: float) -> np.ndarray:
    """x0 F^-1[ gain[alpha, shell(k)] F r_alpha(k) / (E0 + hb2m |k|^2) ]."""
    fk = sfft.fftn(r, axes=(-3, -2, -1), workers=_WORKERS)
    mult = x0 / (e0 + hb2m * g.k2())
    sh = shell_of_modes(g.n)
    fk *= (np.asarray(gain)[:, sh] * mult)[:, None]
    return sfft.ifftn(fk, axes=(-3, -2, -1), workers=_WORKERS)


def shell_steps(r: np.ndarray, g: Grid, hb2m: float, x0: float, e0: float) -> np.ndarray:
    """d[s, alpha] = plain damped residual restricted to shell s."""
    m = r.shape[0]
    out = []
    for s in range(S):
        onehot = np.zeros((m, S))
        onehot[:, s] = 1.0
        out.append(gained_damping(r, onehot, g, hb2m, x0, e0))
    return np.stack(out)


def target_gains(psi: np.ndarray, hpsi: np.ndarray, eps: np.ndarray, mf: MeanField,
                 g: Grid, hb2m: float, x0: float, e0: float, clip: bool = True
                 ) -> np.ndarray:
    """Per state, the real gains minimising |r - sum_s g_s (h - <h>) d_s|^2:
    normal equations (G + lam 1) g = c with G_st = Re<w_s, w_t>,
    c_s = Re<w_s, r>, lam = 1e-6 tr(G) / S, then clamped to [0, GMAX]."""
    r = hpsi - eps[:, None, None, None, None] * psi
    d = shell_steps(r, g, hb2m, x0, e0)
    m = psi.shape[0]
    out = np.zeros((m, S))
    for a in range(m):
        hd = apply_h(d[:, a], mf, g)
        wv = (hd - eps[a] * d[:, a]).reshape(S, -1)
        rv = r[a].reshape(-1)
        G = (wv.conj() @ wv.T).real
        c = (wv.conj() @ rv).real
        lam = 1e-6 * np.trace(G) / S
        gs = np.linalg.solve(G + lam * np.eye(S), c)
        out[a] = np.clip(gs, 0.0, GMAX) if clip else gs
    return out


def init_params(seed: int = 0) -> np.ndarray:
    """Glorot-uniform weights, small positive biases, output bias giving gain 1."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, (fo, fi) in (("W1", (PH, PIN)), ("W2", (PH, PH)), ("W3", (PH, PH))):
        a = math.sqrt(6.0 / (fi + fo))
        p[name] = rng.uniform(-a, a, size=(fo, fi))
    a = math.sqrt(6.0 / (PH + 1))
    p["W4"] = 0.1 * rng.uniform(-a, a, size=PH)
    for b in ("b1", "b2", "b3"):
        p[b] = np.full(PH, 0.01)
    p["b4"] = math.log(1.0 / (GMAX - 1.0))
    return pack(p).astype(np.float32)
