"""Reference of the learned warm start's network (test infrastructure only).

A plain NumPy (FP64) forward and backward pass of the point-set network that the library
evaluates with BF16 MFMA kernels: per-point encoder (3 layers of width 256, ReLU between),
mean pooling of the sources and of the targets into a context vector c = Wc [h_s; h_t] + bc,
per-target head (2 layers) over the target's 8 features whose output is read out against the
context, plus a linear path from the same features: o_j = z2_j . c + ws . f_j + bo, output
centred per instance.  With ``bf16=True`` every operand of a matrix product is rounded
to BF16 (round to nearest even) where it enters the product, as the library does; the
products themselves, biases, activations, pooling and the loss are exact FP64 here (the
library accumulates in FP32); the linear path is FP32 data in FP64 arithmetic here (FP32
arithmetic in the library).  ``bf16=False`` is the plain FP64 network, checked against
finite differences in the tests.  Parameter order and shapes follow ``ibsn_ws_param_count``:
W1 (4 x 256), b1, W2 (256 x 256), b2, W3, b3, Wf (8 x 256), bf, Wg (256 x 256), bg,
Wc (512 x 256), bc, ws (8 x 1), bo.
"""
from __future__ import annotations

import numpy as np

WID, NF, NFH = 256, 4, 8
SHAPES = [("W1", NF, WID), ("b1", 1, WID), ("W2", WID, WID), ("b2", 1, WID), ("W3", WID, WID),
          ("b3", 1, WID), ("Wf", NFH, WID), ("bf", 1, WID), ("Wg", WID, WID), ("bg", 1, WID),
          ("Wc", 2 * WID, WID), ("bc", 1, WID), ("ws", NFH, 1), ("bo", 1, 1)]


def param_count() -> int:
    return sum(r * c for _, r, c in SHAPES)


def unpack(flat: np.ndarray) -> dict:
    out, off = {}, 0
    for name, r, c in SHAPES:
        out[name] = np.asarray(flat[off:off + r * c], dtype=np.float64).reshape(r, c)
        off += r * c
    return out


def pack(d: dict) -> np.ndarray:
    return np.concatenate([d[name].reshape(-1) for name, _, _ in SHAPES])


def bf16_round(x) -> np.ndarray:
    """x rounded to FP32, then to BF16 (round to nearest, ties to even), as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    r = np.where(np.isnan(f), u, r).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def _mm(a, b, rnd):
    if rnd:
        return bf16_round(a) @ bf16_round(b)
    return a @ b


def forward(flat, fs, fte, fth, B, m, n, bf16=True):
    """Outputs o (B n) and the values the backward pass needs.  fs (B m x 4), fte, fth
    (B n x 4) stacked by instance."""
    p = unpack(flat)
    X = np.concatenate([np.asarray(fs, np.float64), np.asarray(fte, np.float64)])
    H1 = np.maximum(_mm(X, p["W1"], bf16) + p["b1"], 0.0)
    H2 = np.maximum(_mm(H1, p["W2"], bf16) + p["b2"], 0.0)
    E = _mm(H2, p["W3"], bf16) + p["b3"]
    hs = E[:B * m].reshape(B, m, WID).mean(1)
    ht = E[B * m:].reshape(B, n, WID).mean(1)
    CTX = np.concatenate([hs, ht], axis=1)
    CB = _mm(CTX, p["Wc"], bf16) + p["bc"]
    XH = np.asarray(fth, np.float64)
    XH32 = np.asarray(fth, np.float32).astype(np.float64)
    Z1 = np.maximum(_mm(XH, p["Wf"], bf16) + p["bf"], 0.0)
    Z2 = np.maximum(_mm(Z1, p["Wg"], bf16) + p["bg"], 0.0)
    O = np.concatenate([_mm(Z2[b * n:(b + 1) * n], CB[b][:, None], bf16).reshape(-1)
                        for b in range(B)]) + p["bo"][0, 0]
    O = O + XH32 @ p["ws"][:, 0]   # linear path in FP32 arithmetic on the FP32 features
    cache = dict(p=p, X=X, H1=H1, H2=H2, E=E, CTX=CTX, CB=CB, XH=XH, Z1=Z1, Z2=Z2)
    return O, cache


def loss(O, target, B, n):
    """Mean over instances and targets of ((o_j - mean o) - t_j)^2."""
    o = O.reshape(B, n)
    oc = o - o.mean(1, keepdims=True)
    return float(((oc - np.asarray(target, np.float64).reshape(B, n)) ** 2).mean())


def loss_and_grad(flat, fs, fte, fth, target, B, m, n, bf16=True):
    """The loss and its gradient with respect to the flat parameters (backpropagation)."""
    O, c = forward(flat, fs, fte, fth, B, m, n, bf16)
    p = c["p"]
    o = O.reshape(B, n)
    d = (o - o.mean(1, keepdims=True)) - np.asarray(target, np.float64).reshape(B, n)
    L = float((d ** 2).mean())
    dO = (2.0 / (B * n)) * (d - d.mean(1, keepdims=True))
    dO = dO.reshape(-1, 1)
    g = {}
    g["bo"] = dO.sum(0, keepdims=True)
    g["ws"] = np.asarray(c["XH"], np.float32).astype(np.float64).T @ dO
    dZ2 = np.zeros_like(c["Z2"])
    dCB = np.zeros_like(c["CB"])
    for b in range(B):
        rows = slice(b * n, (b + 1) * n)
        dZ2[rows] = _mm(dO[rows], c["CB"][b][None, :], bf16)
        dCB[b] = _mm(dO[rows].T, c["Z2"][rows], bf16)[0]
    dZ2 *= c["Z2"] > 0
    g["Wg"] = _mm(c["Z1"].T, dZ2, bf16)
    g["bg"] = dZ2.sum(0, keepdims=True)
    dZ1 = _mm(dZ2, p["Wg"].T, bf16) * (c["Z1"] > 0)
    g["Wf"] = _mm(c["XH"].T, dZ1, bf16)
    g["bf"] = dZ1.sum(0, keepdims=True)
    g["bc"] = dCB.sum(0, keepdims=True)
    g["Wc"] = _mm(c["CTX"].T, dCB, bf16)
    dCTX = _mm(dCB, p["Wc"].T, bf16)
    dE = np.concatenate([np.repeat(dCTX[:, :WID] / m, m, axis=0),
                         np.repeat(dCTX[:, WID:] / n, n, axis=0)])
    g["W3"] = _mm(c["H2"].T, dE, bf16)
    g["b3"] = dE.sum(0, keepdims=True)
    dH2 = _mm(dE, p["W3"].T, bf16) * (c["H2"] > 0)
    g["W2"] = _mm(c["H1"].T, dH2, bf16)
    g["b2"] = dH2.sum(0, keepdims=True)
    dH1 = _mm(dH2, p["W2"].T, bf16) * (c["H1"] > 0)
    g["W1"] = _mm(c["X"].T, dH1, bf16)
    g["b1"] = dH1.sum(0, keepdims=True)
    return L, pack(g), O


GREEN_EPS = (0.01, 0.02, 0.04, 0.08)   # smoothing lengths of the potential features (box units)
KAPPA_PAIRS = 4096                    # (x_i, y_i) pairs that fix the cost's unit


def _images(P, hi):
    """The nine mirror images of the points P (k x 2) in the box [0, hi1] x [0, hi2]:
    reflections across each side and each corner, the point itself included."""
    out = []
    for sx in (-1, 0, 1):
        for sy in (-1, 0, 1):
            Q = P.copy()
            if sx == -1:
                Q[:, 0] = -Q[:, 0]
            elif sx == 1:
                Q[:, 0] = 2.0 * hi[0] - Q[:, 0]
            if sy == -1:
                Q[:, 1] = -Q[:, 1]
            elif sy == 1:
                Q[:, 1] = 2.0 * hi[1] - Q[:, 1]
            out.append(Q)
    return np.concatenate(out)


def green_potentials(xs, ys, a, b, hi, eps=GREEN_EPS):
    """G_k(j) = sum_i a_i g_k(x_i, y_j) - sum_l b_l g_k(y_l, y_j) over the nine images of
    each point, g_k(p, q) = log(|p - q|^2 + eps_k^2) / 2: the free-space Green's function
    of the Laplacian in the plane, smoothed at eps_k, with mirror images for a reflecting
    box.  This is the potential that solves the linearised Monge-Ampere equation
    (Laplacian of the potential = difference of the two densities) for each smoothing.
    Returns (n x len(eps)) in FP64."""
    xi, yi = _images(xs, hi), _images(ys, hi)
    wa = np.tile(np.asarray(a, np.float64), 9)
    wb = np.tile(np.asarray(b, np.float64), 9)
    out = np.zeros((len(ys), len(eps)))
    for j0 in range(0, len(ys), 256):
        yj = ys[j0:j0 + 256]
        dx = ((xi[:, None, :] - yj[None]) ** 2).sum(-1)
        dy = ((yi[:, None, :] - yj[None]) ** 2).sum(-1)
        for k, e in enumerate(eps):
            out[j0:j0 + 256, k] = 0.5 * (wa @ np.log(dx + e * e) - wb @ np.log(dy + e * e))
    return out


def features(x, y, a, b, C):
    """Feature rows of one instance (FP64) and its scale, as defined for ibsn_ws_features.

    Coordinates are taken in the bounding box of all points, shifted to the origin and
    divided by its longer side L.  The cost's unit u = kappa L^2 makes C a function of box
    coordinates, C_ij = u |x~_i - y~_j|^2, with kappa = sum_{i<K} C_ii / sum_{i<K} |x_i - y_i|^2
    over the first K = min(m, n, 4096) pairs.  s = sqrt(mean_j min_i C_ij / u) is the
    typical nearest-source distance in box units, and scale = u s.
      fs  (m x 4) = (x~_i1, x~_i2, m a_i, 1)
      fte (n x 4) = (y~_j1, y~_j2, n b_j, -1)
      fth (n x 8) = (y~_j1, y~_j2, n b_j, min_i C_ij / mean_j min_i C_ij,
                     (G_k(j) - mean_j G_k) / s for the four smoothing lengths)
    """
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    C = np.asarray(C, np.float64)
    m, n = len(a), len(b)
    P = np.concatenate([x, y])
    lo, hi = P.min(0), P.max(0)
    L = float((hi - lo).max())
    L = L if L > 0 else 1.0
    xs, ys = (x - lo) / L, (y - lo) / L
    hin = (hi - lo) / L
    K = min(m, n, KAPPA_PAIRS)
    den = ((x[:K] - y[:K]) ** 2).sum()
    kappa = np.trace(C[:K, :K]) / den if den > 0 else 1.0
    u = kappa * L * L
    cmin = C.min(0)
    cmean = cmin.mean()
    s = np.sqrt(max(cmean / u, 1e-12)) if u > 0 else 1.0
    G = green_potentials(xs, ys, a, b, hin)
    G = (G - G.mean(0)) / s
    fs = np.column_stack([xs[:, 0], xs[:, 1], m * np.asarray(a), np.ones(m)])
    fte = np.column_stack([ys[:, 0], ys[:, 1], n * np.asarray(b), -np.ones(n)])
    fth = np.column_stack([ys[:, 0], ys[:, 1], n * np.asarray(b), cmin / cmean, G])
    return fs, fte, fth, float(u * s)
