"""Grad's tensor Hermite polynomials (test infrastructure only).

Sec. 2.2 expands the distribution in the tensor Hermite polynomials chi^(n)(c)
that are orthogonal under the weight function
omega(c) = (2 pi)^(-D/2) exp(-c^2/2) (eqs. approxf, an). Written out, for
n <= 4 (delta is the Kronecker delta; every index permutation that gives a
distinct term appears once):

    chi^0       = 1
    chi^1_i     = c_i
    chi^2_ij    = c_i c_j - delta_ij
    chi^3_ijk   = c_i c_j c_k - (c_i delta_jk + c_j delta_ik + c_k delta_ij)
    chi^4_ijkl  = c_i c_j c_k c_l
                  - (c_i c_j delta_kl + c_i c_k delta_jl + c_i c_l delta_jk
                     + c_j c_k delta_il + c_j c_l delta_ik + c_k c_l delta_ij)
                  + (delta_ij delta_kl + delta_ik delta_jl + delta_il delta_jk)

They are the Rodrigues derivatives (-1)^n omega^-1 grad^n omega; along one axis
they reduce to the probabilists' polynomials He_n.
"""

import numpy as np


def chi(c, n):
    """chi^(n) evaluated at the rows of c (shape (Q, D)); returns an array of
    shape (Q,) + (D,) * n."""
    c = np.asarray(c, dtype=np.float64)
    Q, D = c.shape
    d = np.eye(D)
    if n == 0:
        return np.ones(Q)
    if n == 1:
        return c.copy()
    if n == 2:
        return np.einsum("qi,qj->qij", c, c) - d[None]
    if n == 3:
        ccc = np.einsum("qi,qj,qk->qijk", c, c, c)
        cd = (np.einsum("qi,jk->qijk", c, d) + np.einsum("qj,ik->qijk", c, d)
              + np.einsum("qk,ij->qijk", c, d))
        return ccc - cd
    if n == 4:
        cccc = np.einsum("qi,qj,qk,ql->qijkl", c, c, c, c)
        ccd = (np.einsum("qi,qj,kl->qijkl", c, c, d)
               + np.einsum("qi,qk,jl->qijkl", c, c, d)
               + np.einsum("qi,ql,jk->qijkl", c, c, d)
               + np.einsum("qj,qk,il->qijkl", c, c, d)
               + np.einsum("qj,ql,ik->qijkl", c, c, d)
               + np.einsum("qk,ql,ij->qijkl", c, c, d))
        dd = (np.einsum("ij,kl->ijkl", d, d) + np.einsum("ik,jl->ijkl", d, d)
              + np.einsum("il,jk->ijkl", d, d))
        return cccc - ccd + dd[None]
    raise ValueError("chi^(n) is provided for n <= 4")


def basis(c, N):
    """[chi^(0), ..., chi^(N)] at the rows of c."""
    return [chi(c, n) for n in range(N + 1)]


def contract(a, x):
    """Full contraction a : x over the trailing tensor indices. a has shape
    (M,) + (D,)*n (one coefficient tensor per cell), x has shape
    (Q,) + (D,)*n (one basis tensor per velocity); the result is (Q, M)."""
    n = a.ndim - 1
    if n == 0:
        return np.multiply.outer(x, a)
    M = a.shape[0]
    Q = x.shape[0]
    return x.reshape(Q, -1) @ a.reshape(M, -1).T
