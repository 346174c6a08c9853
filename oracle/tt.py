"""Oracle: tensor-train (TT) algebra for 3-way tensors (time x chaos x space).

Test infrastructure only (see oracle/__init__.py).

Paper convention (sec. 4.1, eq. 4.1-4.2): a TT is (G1, G2, G3) with
G1 (n1 x r1), G2 (r1 x n2 x r2), G3 (r2 x n3) and
z(i1,i2,i3) = sum_{a,b} G1[i1,a] G2[a,i2,b] G3[b,i3];
vec index i3 + i2*n3 + i1*n2*n3, i.e. numpy C-order reshape of (n1,n2,n3).

* tt_svd      Alg. 4.1 (TT-SVD of a full tensor), delta = eps*||z||/sqrt(d-1).
* tt_round    truncation T_eps of a TT (eq. 4.5-4.7): right-to-left QR
              orthogonalization, then left-to-right truncated SVDs with the same
              delta (the procedure sec. 4.1 refers to for TT input).
* concat      sum of TTs by core concatenation (ranks add, sec. 4.1).
* tt_dot      inner product by left-to-right contraction.
* kron_apply  (X1 (x) X2 (x) X3) z applied core by core (eq. 4.4).

Pins (tests/test_oracle_tt.py): tt_round reproduces TT-SVD of the full tensor
(ranks and error), the truncation error obeys eq. 4.7 and equals the discarded
singular values (Eckart-Young) per unfolding; kron_apply equals an explicit
scipy.sparse.kron matvec; tt_dot equals the dot of the full vectors.
"""
from __future__ import annotations

import numpy as np


def full(t):
    G1, G2, G3 = t
    return np.einsum("ia,ajb,bk->ijk", G1, G2, G3, optimize=True)


def ranks(t):
    return t[0].shape[1], t[2].shape[0]


def rank_cut(s: np.ndarray, delta: float) -> int:
    """Smallest r >= 1 such that the discarded tail sqrt(sum_{i>r} s_i^2) <= delta
    (Alg. 4.1 line 4; ties keep the smaller rank)."""
    tail2 = np.concatenate([np.cumsum((s ** 2)[::-1])[::-1], [0.0]])
    for r in range(1, s.size + 1):
        if tail2[r] <= delta * delta:
            return r
    return max(1, s.size)


def tt_svd(X: np.ndarray, eps: float):
    """Alg. 4.1 with d = 3, delta_j = eps ||X||_F / sqrt(2)."""
    n1, n2, n3 = X.shape
    delta = eps * np.linalg.norm(X) / np.sqrt(2.0)
    U, s, Vt = np.linalg.svd(X.reshape(n1, n2 * n3), full_matrices=False)
    r1 = rank_cut(s, delta)
    G1 = U[:, :r1]
    Z = (s[:r1, None] * Vt[:r1]).reshape(r1 * n2, n3)
    U, s, Vt = np.linalg.svd(Z, full_matrices=False)
    r2 = rank_cut(s, delta)
    G2 = U[:, :r2].reshape(r1, n2, r2)
    G3 = s[:r2, None] * Vt[:r2]
    return G1, G2, G3


def orthogonalize_rl(t):
    """Right-to-left QR sweep: returns an equal TT whose cores 2 and 3 are
    right-orthonormal; its norm is ||G1||_F."""
    G1, G2, G3 = t
    r1, n2, r2 = G2.shape
    Q, R = np.linalg.qr(G3.T)                 # G3^T = Q R
    G3n = Q.T
    G2 = np.einsum("aib,cb->aic", G2, R)      # G2 x_3 R^T
    r2n = G3n.shape[0]
    Q2, R2 = np.linalg.qr(G2.reshape(r1, n2 * r2n).T)
    G2n = Q2.T.reshape(-1, n2, r2n)
    G1n = G1 @ R2.T
    return G1n, G2n, G3n


def tt_norm(t) -> float:
    return float(np.linalg.norm(orthogonalize_rl(t)[0]))


def tt_round(t, eps: float, max_rank: int | None = None):
    """T_eps: ||round(z) - z||_F <= eps ||z||_F (eq. 4.6).  Output is
    left-orthonormal (G1, G2 orthonormal; G3 carries the norm)."""
    G1, G2, G3 = orthogonalize_rl(t)
    nrm = np.linalg.norm(G1)
    delta = eps * nrm / np.sqrt(2.0)
    r1, n2, r2 = G2.shape
    U, s, Vt = np.linalg.svd(G1, full_matrices=False)
    k1 = rank_cut(s, delta)
    G1 = U[:, :k1]
    G2 = np.einsum("ab,bic->aic", s[:k1, None] * Vt[:k1], G2)
    U, s, Vt = np.linalg.svd(G2.reshape(k1 * n2, r2), full_matrices=False)
    k2 = rank_cut(s, delta)
    if max_rank is not None and max(k1, k2) > max_rank:
        raise ValueError("rank capacity exceeded")
    G2 = U[:, :k2].reshape(k1, n2, k2)
    G3 = (s[:k2, None] * Vt[:k2]) @ G3
    return G1, G2, G3


def concat(tts, coefs=None):
    """sum_i coefs[i] * tts[i] as one TT (core concatenation; ranks add).
    Scalars are folded into core 1."""
    if coefs is None:
        coefs = [1.0] * len(tts)
    n2 = tts[0][1].shape[1]
    R1 = sum(t[0].shape[1] for t in tts)
    R2 = sum(t[2].shape[0] for t in tts)
    G1 = np.concatenate([c * t[0] for c, t in zip(coefs, tts)], axis=1)
    G2 = np.zeros((R1, n2, R2))
    G3 = np.concatenate([t[2] for t in tts], axis=0)
    a = b = 0
    for t in tts:
        ra, rb = t[0].shape[1], t[2].shape[0]
        G2[a:a + ra, :, b:b + rb] = t[1]
        a += ra
        b += rb
    return G1, G2, G3


def scale(t, c):
    return c * t[0], t[1], t[2]


def tt_dot(x, y) -> float:
    W = x[0].T @ y[0]
    W = np.einsum("aib,ac,cid->bd", x[1], W, y[1], optimize=True)
    return float(np.sum(W * (x[2] @ y[2].T)))


def mode_apply(t, X1=None, X2=None, X3=None):
    """One Kronecker term (X1 (x) X2 (x) X3) applied to a TT (eq. 4.4): the
    result has the same ranks.  Each X may be None (identity), a dense or
    sparse matrix."""
    G1, G2, G3 = t
    if X1 is not None:
        G1 = X1 @ G1
    if X2 is not None:
        G2 = np.einsum("ij,ajb->aib", np.asarray(X2), G2)
    if X3 is not None:
        G3 = np.asarray((X3 @ G3.T)).T
    return G1, G2, G3


def kron_apply(terms, t):
    """sum_k (X1_k (x) X2_k (x) X3_k) t, each term applied by mode_apply and the
    results concatenated."""
    return concat([mode_apply(t, *term) for term in terms])


# ---- pairs (velocity TT, pressure TT): u and p are separate tensor trains
# (Alg. 4.2 discussion: truncation applies to du and dp separately) ----

def pair_dot(x, y):
    return tt_dot(x[0], y[0]) + tt_dot(x[1], y[1])


def pair_norm(x):
    return float(np.sqrt(tt_norm(x[0]) ** 2 + tt_norm(x[1]) ** 2))


def pair_round(x, eps):
    return tt_round(x[0], eps), tt_round(x[1], eps)


def pair_concat(xs, coefs=None):
    return concat([x[0] for x in xs], coefs), concat([x[1] for x in xs], coefs)


def pair_scale(x, c):
    return scale(x[0], c), scale(x[1], c)


def pair_full(x):
    return np.concatenate([full(x[0]).ravel(), full(x[1]).ravel()])


def zero_tt(n1, n2, n3):
    return np.zeros((n1, 1)), np.zeros((1, n2, 1)), np.zeros((1, n3))
