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
  * the leading left singular vectors of each iteration's I x R^(m-1)
    unfolding come from its small Gram matrix: formed in double precision on
    the device, eigendecomposed on the host, mapped back through the unfolding
    and re-orthonormalized by one Cholesky pass (a tall-skinny SVD on the device
    costs milliseconds; this is one product and a few small host factorizations).
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
    Q = _orth(Y)
    for _ in range(power):
        Z = torch.conj(hankel_matmat(h, torch.conj(Q), cols, rows))  # A^H Q
        Z = _orth(Z)
        Q = _orth(hankel_matmat(h, Z, rows, cols))
    # B = Q^H A (k x cols) = (A^H Q)^H; the left singular vectors of A are Q times
    # those of B, the eigenvectors of B B^H = (A^H Q)^H (A^H Q) (k x k)
    BH = _wide(torch.conj(hankel_matmat(h, torch.conj(Q), cols, rows)))  # A^H Q, shape (cols, k)
    _, Vb = torch.linalg.eigh(_cross(BH, BH))
    Ub = Vb.flip(1)[:, :rank].to(Q.dtype).to(Q.device)
    return Q @ Ub


def _wide(t: torch.Tensor) -> torch.Tensor:
    return t.to(torch.complex128 if t.is_complex() else torch.float64)


def _cross(A: torch.Tensor, B: torch.Tensor, blocks: int = 64) -> torch.Tensor:
    """A^H B for tall A (n x a) and B (n x b), on the host: the n rows split
    into `blocks` slabs multiplied in one batched product and summed (a plain
    product with an n-long inner dimension and a tiny output runs on a handful
    of workgroups)."""
    n = A.shape[0]
    pad = (-n) % blocks
    if pad:
        A = torch.cat([A, A.new_zeros(pad, A.shape[1])])
        B = torch.cat([B, B.new_zeros(pad, B.shape[1])])
    As = A.reshape(blocks, -1, A.shape[1])
    Bs = B.reshape(blocks, -1, B.shape[1])
    return torch.bmm(As.conj().transpose(1, 2).contiguous(), Bs.contiguous()).sum(0).cpu()


def _orth(Y: torch.Tensor) -> torch.Tensor:
    """Orthonormal basis of the columns of a tall Y: two Cholesky QR passes in
    double precision (Y <- Y L^{-H}, L L^H = Y^H Y); the device QR where the
    Gram matrix is not numerically positive definite or orthogonality is lost."""
    Yd = _wide(Y)
    for _ in range(2):
        L, info = torch.linalg.cholesky_ex(_cross(Yd, Yd))
        if int(info) != 0:
            return torch.linalg.qr(Y)[0]
        Yd = Yd @ torch.linalg.inv(L).conj().t().to(Y.device)
    eye = torch.eye(Yd.shape[1], dtype=Yd.dtype)
    if float((_cross(Yd, Yd) - eye).abs().max()) > 1e-10:
        return torch.linalg.qr(Y)[0]
    return Yd.to(Y.dtype)


def leading_left(M: torch.Tensor, rank: int) -> torch.Tensor:
    """The `rank` leading left singular vectors of a tall matrix M (n x k, k
    small), in M's dtype: v_j, s_j^2 from the eigenpairs of the k x k Gram
    matrix M^H M (double precision), u_j = M v_j / s_j, then one Cholesky
    re-orthonormalization (U <- U L^{-H}, L L^H = U^H U) in double precision."""
    Md = _wide(M)
    G = _cross(Md, Md)
    w, V = torch.linalg.eigh(G)                      # ascending eigenvalues
    w = w.flip(0)[:rank].clamp_min(float(w[-1]) * 1e-30 + 1e-300)
    V = V.flip(1)[:, :rank]
    U = Md @ (V / torch.sqrt(w)).to(M.device)
    L = torch.linalg.cholesky(_cross(U, U))
    U = U @ torch.linalg.inv(L).conj().t().to(M.device)
    return U.to(M.dtype)


def unfold1(h: torch.Tensor, U: torch.Tensor, m: int) -> torch.Tensor:
    """Unfold_1(H x_2 conj(U) ... x_m conj(U)) as an n x R^(m-1) matrix."""
    T = _b.hankel_tensor_matrix(h, torch.conj(U), m)
    n = U.shape[0]
    return T.permute([0] + list(range(m - 1, 0, -1))).reshape(n, -1)


def hooi(h: torch.Tensor, m: int, rank: int, iters: int = 10, tol: float = 0.0,
         U0: Optional[torch.Tensor] = None, seed: int = 0):
    """Algorithm 4.2.  Returns (U, S, history): U (n x rank) with orthonormal
    columns, the core S = H conj(U)^m of shape (rank,)*m, and the subspace change
    1 - sigma_min(U_old^H U_new) of each iteration (with tol > 0 it stops once the
    change falls below tol)."""
    n = (h.numel() + m - 1) // m
    if m * (n - 1) + 1 != h.numel():
        raise ValueError("h must have m(n-1)+1 entries for a square order-m Hankel tensor")
    U = hankel_leading_subspace(h, n, rank, seed=seed) if U0 is None else U0
    history = []
    for _ in range(iters):
        M = unfold1(h, U, m)
        Un = leading_left(M, rank)
        overlap = _cross(_wide(U), _wide(Un))
        change = max(0.0, 1.0 - float(torch.linalg.svdvals(overlap).min()))
        history.append(change)
        U = Un
        if tol > 0 and change < tol:
            break
    # core: S[j1, j2..jm] = sum_i conj(U)[i, j1] (H x_2 conj(U) ... x_m conj(U))[i, j2..jm]
    M = unfold1(h, U, m)
    S = (torch.conj(U).t() @ M).reshape([rank] * m)
    S = S.permute([0] + list(range(m - 1, 0, -1)))
    return U, S, history
