"""The blocking scheme of the GPU band reduction, written out in numpy at small
sizes and checked against the band oracle: panels factored as sub-panels whose
block reflectors update the rest of the panel, T assembled blockwise as
T[0:j0, j] = -T[0:j0, 0:j0] (V[:, 0:j0]^T V_j) T_j, the left update
C -= V T^T V^T C, the row panel factored as the QR of its transpose and the
right update D -= D V T V^T.  This pins the algebra the executor relies on
(which T, which side, which transpose) independently of the GPU; the GPU path
itself is compared with the oracle in test_gpu_band.py."""
import numpy as np
import pytest

import oracle
import synth


def _geqr2(P):
    """Column-by-column Householder QR in place (larfg convention); returns tau."""
    m, w = P.shape
    tau = np.zeros(w)
    for j in range(w):
        alpha = P[j, j]
        s = float(np.dot(P[j + 1:, j], P[j + 1:, j]))
        if s == 0.0:
            continue
        beta = -np.sqrt(alpha * alpha + s) if alpha >= 0.0 else np.sqrt(alpha * alpha + s)
        tau[j] = (beta - alpha) / beta
        P[j + 1:, j] *= 1.0 / (alpha - beta)
        P[j, j] = beta
        v = np.concatenate(([1.0], P[j + 1:, j]))
        P[j:, j + 1:] -= tau[j] * np.outer(v, v @ P[j:, j + 1:])
    return tau


def _v_of(P):
    m, w = P.shape
    V = np.tril(P[:, :w], -1)
    V[np.arange(w), np.arange(w)] = 1.0
    return V


def _larft(V, tau):
    """T of I - V T V^T = H_0 H_1 ... column by column (the reference)."""
    w = V.shape[1]
    T = np.zeros((w, w))
    for j in range(w):
        T[:j, j] = -tau[j] * T[:j, :j] @ (V[:, :j].T @ V[:, j])
        T[j, j] = tau[j]
    return T


def _panel_blocked(P, sub):
    """The executor's wide-panel scheme: returns (tau, T); P becomes R and V."""
    m, pw = P.shape
    tau = np.zeros(pw)
    T = np.zeros((pw, pw))
    for j0 in range(0, pw, sub):
        jw = min(sub, pw - j0)
        Pj = P[j0:, j0:j0 + jw]
        tau[j0:j0 + jw] = _geqr2(Pj)
        Vj = _v_of(Pj)
        Tj = _larft(Vj, tau[j0:j0 + jw])
        T[j0:j0 + jw, j0:j0 + jw] = Tj
        if j0 > 0:
            Vprev = P[j0:, :j0]                  # rows >= j0 of the earlier sub-panels: all below their diagonal
            T[:j0, j0:j0 + jw] = -T[:j0, :j0] @ (Vprev.T @ Vj) @ Tj
        C = P[j0:, j0 + jw:]
        C -= Vj @ (Tj.T @ (Vj.T @ C))
    return tau, T


def _band_blocked(A, w, sub):
    A = np.array(A, dtype=np.float64, order="F", copy=True)
    n = A.shape[0]
    tauq, taup = np.zeros(n), np.zeros(n)
    for k in range(0, n, w):
        kw = min(w, n - k)
        tq, T = _panel_blocked(A[k:, k:k + kw], sub)
        tauq[k:k + kw] = tq
        V = _v_of(A[k:, k:k + kw])
        C = A[k:, k + kw:]
        C -= V @ (T.T @ (V.T @ C))                 # left: C <- (I - V T V^T)^T C
        c0 = k + w
        if c0 >= n:
            continue
        npn = n - c0
        wp = min(kw, npn)
        Z = np.array(A[k:k + wp, c0:].T, order="F")
        tp, T2 = _panel_blocked(Z, sub)
        taup[k:k + wp] = tp
        A[k:k + wp, c0:] = Z.T
        V2 = _v_of(Z)
        D = A[k + wp:, c0:]
        D -= (D @ V2) @ T2 @ V2.T                  # right: D <- D (I - V T V^T)
    return A, tauq, taup


@pytest.mark.parametrize("m,pw,sub", [(40, 12, 4), (33, 10, 4), (25, 9, 3)])
def test_blocked_panel_equals_unblocked(m, pw, sub):
    A = synth.uniform(m, seed=m + pw)[:, :pw].copy(order="F")
    P1 = A.copy(order="F")
    tau1 = _geqr2(P1)
    T1 = _larft(_v_of(P1), tau1)
    P2 = A.copy(order="F")
    tau2, T2 = _panel_blocked(P2, sub)
    assert np.abs(P2 - P1).max() <= 1e-13
    assert np.abs(tau2 - tau1).max() <= 1e-14
    assert np.abs(T2 - T1).max() <= 1e-13


@pytest.mark.parametrize("n,w,sub", [(30, 6, 2), (40, 12, 4), (37, 12, 5), (26, 30, 8)])
def test_blocked_band_equals_oracle(n, w, sub):
    A = synth.uniform(n, seed=3 * n + w)
    F, tq, tp = _band_blocked(A, w, sub)
    oF, otq, otp = oracle.gebrd_band(A, w)
    assert np.abs(F - oF).max() <= 1e-12
    assert np.abs(tq - otq).max() <= 1e-13
    assert np.abs(tp - otp).max() <= 1e-13


def test_wrong_t_block_sign_is_caught():
    """A plausible slip in the T assembly (the sign of the block above T_j)
    breaks the equality with the unblocked T."""
    A = synth.uniform(40, seed=4)[:, :12].copy(order="F")
    P = A.copy(order="F")
    tau, T = _panel_blocked(P, 4)
    Tref = _larft(_v_of(P), tau)
    Tbad = T.copy()
    Tbad[:4, 4:8] = -Tbad[:4, 4:8]
    assert np.abs(T - Tref).max() <= 1e-13
    assert np.abs(Tbad - Tref).max() > 1e-3
