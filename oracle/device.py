"""Block-tridiagonal open-system matrix and its Green's-function columns.

Test infrastructure only (see the package docstring).

The device has N slabs of m basis functions; the Galerkin matrices are
block tridiagonal (Sec. "Matrix equations", eq. infinite_system).  With the
extrinsic potential projected on the linear shape functions the open
system matrix A(z) = zS - H - H_ext - Sigma has the blocks

    A_ii      = (z - Vd_i) Sd_i - Hd_i        (minus Sigma_L at i = 0 and
                                               Sigma_R at i = N-1)
    A_{i,i+1} = (z - Vu_i) Su_i - Hu_i
    A_{i+1,i} = (z - Vu_i) Su_i^H - Hu_i^H

(eq. qtbm_system: [EM - H - Sigma] c = B).  G = A^-1; only the first and the
last block columns are needed for transmission and density.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

POT_DIAG = 0
POT_LINEAR_FE = 1


def potential_weights(V, VL, VR, mode):
    """Weights Vd (N,), Vu (N-1,) of the overlap blocks in H_ext.

    DIAG: H_ext adds V_i S_ii on the diagonal only.
    LINEAR_FE: the potential is linear between nodes, V(z) = sum_k V_k
    f_k(z), and the extrinsic matrix element over the hat functions f_i f_j
    (Sec. "Matrix equations", V^e element) is taken as V-bar times the
    overlap block, with V-bar the shape-function-weighted average:
    int f_i^3 = 1/2, int f_i^2 f_{i+-1} = 1/12, int f_i^2 = 2/3 and
    int f_i f_{i+1} = 1/6 give Vd_i = 3/4 V_i + (V_{i-1} + V_{i+1}) / 8 and
    Vu_i = (V_i + V_{i+1}) / 2, with V_{-1} = VL and V_N = VR."""
    V = np.asarray(V, dtype=np.float64)
    N = V.shape[0]
    if mode == POT_DIAG:
        return V.copy(), np.zeros(max(N - 1, 0))
    if mode != POT_LINEAR_FE:
        raise ValueError("unknown potential mode")
    ext = np.concatenate([[VL], V, [VR]])
    Vd = 0.75 * ext[1:-1] + 0.125 * (ext[:-2] + ext[2:])
    Vu = 0.5 * (V[:-1] + V[1:])
    return Vd, Vu


def assemble(z, Hd, Hu, Sd, Su, Vd, Vu):
    """Diagonal, upper and lower blocks of zS - H - H_ext (no Sigma)."""
    Ad = (z - Vd)[:, None, None] * Sd - Hd
    Au = (z - Vu)[:, None, None] * Su - Hu
    SuH = np.swapaxes(Su.conj(), -1, -2)
    HuH = np.swapaxes(Hu.conj(), -1, -2)
    Al = (z - Vu)[:, None, None] * SuH - HuH
    return Ad, Au, Al


def first_block_column(Ad, Au, Al):
    """G_{:,0} by elimination from the right end (right-connected sweep).

    gR_{N-1} = A_{N-1,N-1}^-1, gR_i = (A_ii - A_{i,i+1} gR_{i+1} A_{i+1,i})^-1,
    then G_00 = gR_0 and G_{i+1,0} = -gR_{i+1} A_{i+1,i} G_{i,0}."""
    N = Ad.shape[0]
    gR = [None] * N
    gR[N - 1] = np.linalg.inv(Ad[N - 1])
    for i in range(N - 2, -1, -1):
        gR[i] = np.linalg.inv(Ad[i] - Au[i] @ gR[i + 1] @ Al[i])
    G = np.empty_like(Ad)
    G[0] = gR[0]
    for i in range(N - 1):
        G[i + 1] = -gR[i + 1] @ (Al[i] @ G[i])
    return G


def last_block_column(Ad, Au, Al):
    """G_{:,N-1}: the first block column of the block-reversed system."""
    G = first_block_column(Ad[::-1], Al[::-1], Au[::-1])
    return G[::-1]


def columns_two_pass(Ad, Au, Al):
    """G_{:,0} and G_{:,N-1} in the other order: left-connected forward
    factorisation D_i = A_ii - A_{i,i-1} D_{i-1}^-1 A_{i-1,i}, forward
    substitution for the first column, then back substitution."""
    N, m = Ad.shape[0], Ad.shape[1]
    Dinv = [None] * N
    X = [None] * N
    Z = [None] * N
    D = Ad[0].copy()
    y = np.eye(m, dtype=np.complex128)
    for i in range(N):
        if i > 0:
            D = Ad[i] - Al[i - 1] @ X[i - 1]
            y = -Al[i - 1] @ Z[i - 1]
        Dinv[i] = np.linalg.inv(D)
        Z[i] = Dinv[i] @ y
        if i < N - 1:
            X[i] = Dinv[i] @ Au[i]
    G0 = np.empty_like(Ad)
    GN = np.empty_like(Ad)
    G0[N - 1] = Z[N - 1]
    GN[N - 1] = Dinv[N - 1]
    for i in range(N - 2, -1, -1):
        G0[i] = Z[i] - X[i] @ G0[i + 1]
        GN[i] = -X[i] @ GN[i + 1]
    return G0, GN


def full_matrix(Ad, Au, Al):
    N, m = Ad.shape[0], Ad.shape[1]
    A = np.zeros((N * m, N * m), dtype=np.complex128)
    for i in range(N):
        A[i * m:(i + 1) * m, i * m:(i + 1) * m] = Ad[i]
        if i < N - 1:
            A[i * m:(i + 1) * m, (i + 1) * m:(i + 2) * m] = Au[i]
            A[(i + 1) * m:(i + 2) * m, i * m:(i + 1) * m] = Al[i]
    return A


def columns_dense(Ad, Au, Al):
    """Brute force: the full inverse of A (tiny systems only)."""
    N, m = Ad.shape[0], Ad.shape[1]
    G = np.linalg.inv(full_matrix(Ad, Au, Al))
    G0 = G[:, :m].reshape(N, m, m)
    GN = G[:, (N - 1) * m:].reshape(N, m, m)
    return G0, GN


def columns_banded(Ad, Au, Al):
    """LAPACK banded LU with partial pivoting (zgbsv via solve_banded) on
    A, with bandwidth 2m-1 on each side, for both block columns."""
    N, m = Ad.shape[0], Ad.shape[1]
    n = N * m
    bw = 2 * m - 1
    ab = np.zeros((2 * bw + 1, n), dtype=np.complex128)
    A = full_matrix(Ad, Au, Al) if n <= 4096 else None
    if A is not None:
        for d in range(-min(bw, n - 1), min(bw, n - 1) + 1):
            diag = np.diagonal(A, d)
            if d >= 0:
                ab[bw - d, d:] = diag
            else:
                ab[bw - d, :n + d] = diag
    else:
        for i in range(N):
            blocks = [(i, Ad[i])]
            if i < N - 1:
                blocks.append((i + 1, Au[i]))
            if i > 0:
                blocks.append((i - 1, Al[i - 1]))
            for j, blk in blocks:
                for r in range(m):
                    rows = i * m + r
                    cols = j * m + np.arange(m)
                    ab[bw + rows - cols, cols] = blk[r]
    rhs = np.zeros((n, 2 * m), dtype=np.complex128)
    rhs[:m, :m] = np.eye(m)
    rhs[n - m:, m:] = np.eye(m)
    sol = scipy.linalg.solve_banded((bw, bw), ab, rhs)
    return sol[:, :m].reshape(N, m, m), sol[:, m:].reshape(N, m, m)
