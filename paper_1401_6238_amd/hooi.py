"""Best rank-(R, ..., R) approximation of a square Hankel tensor by higher-order
orthogonal iteration (Section 4.2, Algorithm 4.2 for square Hankel tensors,
where U_1 = ... = U_m = U).

Every product with the tensor goes through the library's fast Hankel
products on the GPU:
  * the initial U, the R leading left singular vectors of the I x (d_H - I + 1)
    Hankel matrix of h (the mode-1 unfolding with its redundant columns
    removed), comes from a randomized range finder with power iterations whose
    matrix-vector products are order-2 Hankel tensor-vector products (the
    matrix is never formed);
  * each iteration's Unfold_1(H x_2 conj(U) ... x_m conj(U)) is one Hankel
    tensor-matrix product (hankel_tensor_matrix);
  * the small dense factorizations (QR, SVD of an I x R^(m-1) matrix) use
    torch.linalg on the same device.
"""
from __future__ import annotations

from typing import Optional

import torch

from . import binding as _b


def hankel_matmat(h: torch.Tensor, X: torch.Tensor, rows: int, cols: int) -> torch.Tensor:
    """A @ X for the rows x cols Hankel matrix A[i, j] = h[i + j] (len(h) = rows +
    cols - 1) and X of shape (cols, k): k order-2 tensor-vector products in one
    grouped batch."""
    k = X.shape[1]
    X = X.resolve_conj().resolve_neg()
    items = [{"m": 2, "dims": [rows, cols], "h": h, "vectors": [None, X[:, j].contiguous()]} for j in range(k)]
    plan = _b.Plan(items)
    try:
        outs = plan.execute()
        plan.status()
    finally:
        plan.close()
    return torch.stack([y for y, _ in outs], dim=1)


def hankel_leading_subspace(h: torch.Tensor, rows: int, rank: int, oversample: int = 8, power: int = 4,
                            seed: int = 0) -> torch.Tensor:
    """R leading left singular vectors of the rows x (len(h) - rows + 1) Hankel
    matrix of h, by a randomized range finder with `power` power iterations
    (A^H y = conj(A^T conj(y)), and A^T is the Hankel matrix of h transposed)."""
    cols = h.numel() - rows + 1
    k = rank + oversample
    g = torch.Generator(device="cpu").manual_seed(seed)
    omega = torch.randn(cols, k, generator=g, dtype=torch.float64)
    omega = omega.to(h.dtype).to(h.device)
    Y = hankel_matmat(h, omega, rows, cols)
    Q, _ = torch.linalg.qr(Y)
    for _ in range(power):
        Z = torch.conj(hankel_matmat(h, torch.conj(Q), cols, rows))  # A^H Q
        Z, _ = torch.linalg.qr(Z)
        Q, _ = torch.linalg.qr(hankel_matmat(h, Z, rows, cols))
    # B = Q^H A (k x cols) = (A^H Q)^H; left singular vectors of A = Q (left sv of B)
    BH = torch.conj(hankel_matmat(h, torch.conj(Q), cols, rows))  # A^H Q, shape (cols, k)
    Ub, _, _ = torch.linalg.svd(BH.conj().t(), full_matrices=False)
    return (Q @ Ub)[:, :rank]


def unfold1(h: torch.Tensor, U: torch.Tensor, m: int) -> torch.Tensor:
    """Unfold_1(H x_2 conj(U) ... x_m conj(U)) as an n x R^(m-1) matrix."""
    T = _b.hankel_tensor_matrix(h, torch.conj(U), m)
    n = U.shape[0]
    return T.permute([0] + list(range(m - 1, 0, -1))).reshape(n, -1)


def hooi(h: torch.Tensor, m: int, rank: int, iters: int = 10, tol: float = 0.0,
         U0: Optional[torch.Tensor] = None, seed: int = 0):
    """Algorithm 4.2.  Returns (U, S, history): U (n x rank) with orthonormal
    columns, the core S = H conj(U)^m of shape (rank,)*m, and the subspace change
    1 - sigma_min(U_old^H U_new) of each iteration (stops early below tol)."""
    n = (h.numel() + m - 1) // m
    if m * (n - 1) + 1 != h.numel():
        raise ValueError("h must have m(n-1)+1 entries for a square order-m Hankel tensor")
    U = hankel_leading_subspace(h, n, rank, seed=seed) if U0 is None else U0
    history = []
    for _ in range(iters):
        M = unfold1(h, U, m)
        Un, _, _ = torch.linalg.svd(M, full_matrices=False)
        Un = Un[:, :rank]
        change = 1.0 - float(torch.linalg.svdvals(U.conj().t() @ Un).min())
        history.append(change)
        U = Un
        if change < tol:
            break
    # core: S[j1, j2..jm] = sum_i conj(U)[i, j1] (H x_2 conj(U) ... x_m conj(U))[i, j2..jm]
    M = unfold1(h, U, m)
    S = (torch.conj(U).t() @ M).reshape([rank] * m)
    S = S.permute([0] + list(range(m - 1, 0, -1)))
    return U, S, history
