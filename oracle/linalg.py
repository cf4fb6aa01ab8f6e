"""CPU FP64 oracle -- sparse SPD factorisation without the BTA structure.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in
``oracle/``.

The quantities the method needs from a precision matrix Q -- log|Q| from the
diagonal of its Cholesky factor (Eq. 1), the solution of Q x = r (the mean of
p_G, Eq. 3) and selected entries of Q^{-1} (the marginal variances, Section
III, selected inversion) -- have plain definitions that any Cholesky of Q
reaches up to rounding.  Two routes are provided:

* ``DenseSPD``: numpy/LAPACK dense Cholesky, for small N.
* ``BandedSPD``: a generic reverse Cuthill-McKee ordering of the sparse part,
  LAPACK banded Cholesky (dpbtrf via scipy), and a bordered Schur complement
  for the trailing dense rows (the fixed effects), for large N.

Neither knows about time steps, blocks or arrowheads.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
from scipy.sparse.csgraph import reverse_cuthill_mckee


class NotSPD(Exception):
    pass


class DenseSPD:
    """Dense Cholesky Q = L L^T of a (sparse or dense) SPD matrix."""

    def __init__(self, Q):
        Qd = Q.toarray() if sp.issparse(Q) else np.asarray(Q, np.float64)
        self.N = Qd.shape[0]
        try:
            self.L = np.linalg.cholesky(Qd)
        except np.linalg.LinAlgError as e:
            raise NotSPD(str(e))

    def logdet(self) -> float:
        return float(2.0 * np.sum(np.log(np.diag(self.L))))

    def solve(self, r):
        return sla.cho_solve((self.L, True), r)

    def inv_diag(self, idx=None):
        Linv = sla.solve_triangular(self.L, np.eye(self.N), lower=True)
        d = np.sum(Linv * Linv, axis=0)      # diag(L^-T L^-1)
        return d if idx is None else d[np.asarray(idx)]


class BandedSPD:
    """Cholesky of Q = [[Q11, Q12], [Q21, Q22]] with Q11 sparse (banded after
    a reverse Cuthill-McKee ordering) and Q22 a small dense border of size
    ``a``:  log|Q| = log|Q11| + log|S|,  S = Q22 - Q21 Q11^{-1} Q12."""

    def __init__(self, Q, a: int):
        Q = sp.csr_matrix(Q)
        N = Q.shape[0]
        n1 = N - a
        self.N, self.n1, self.a = N, n1, a
        Q11 = Q[:n1, :n1].tocsr()
        perm = reverse_cuthill_mckee(Q11, symmetric_mode=True)
        self.perm = perm.astype(np.int64)
        Q11p = Q11[perm][:, perm].tocoo()
        low = Q11p.row >= Q11p.col
        ri, ci, vv = Q11p.row[low], Q11p.col[low], Q11p.data[low]
        kd = int(np.max(ri - ci)) if ri.size else 0
        self.kd = kd
        ab = np.zeros((kd + 1, n1))
        ab[ri - ci, ci] = vv
        try:
            self.cb = sla.cholesky_banded(ab, lower=True, overwrite_ab=True,
                                          check_finite=False)
        except np.linalg.LinAlgError as e:
            raise NotSPD(str(e))
        del ab
        if a > 0:
            Q12 = Q[:n1, n1:].toarray()[perm]       # rows in RCM order
            Q22 = Q[n1:, n1:].toarray()
            Y = self._solve11(Q12)
            S = Q22 - Q12.T @ Y
            self.Q12p = Q12
            try:
                self.Ls = np.linalg.cholesky(S)
            except np.linalg.LinAlgError as e:
                raise NotSPD(str(e))
        else:
            self.Q12p = np.zeros((n1, 0))
            self.Ls = np.zeros((0, 0))

    def _solve11(self, rhs_perm):
        return sla.cho_solve_banded((self.cb, True), rhs_perm,
                                    check_finite=False)

    def logdet(self) -> float:
        ld = 2.0 * np.sum(np.log(self.cb[0]))
        if self.a:
            ld += 2.0 * np.sum(np.log(np.diag(self.Ls)))
        return float(ld)

    def solve(self, r):
        """Q x = r by block elimination on the border."""
        r = np.asarray(r, np.float64)
        one = r.ndim == 1
        R = r[:, None] if one else r
        r1 = R[:self.n1][self.perm]
        r2 = R[self.n1:]
        y1 = self._solve11(r1)
        if self.a:
            rhs2 = r2 - self.Q12p.T @ y1
            x2 = sla.cho_solve((self.Ls, True), rhs2)
            x1p = self._solve11(r1 - self.Q12p @ x2)
        else:
            x2 = r2
            x1p = y1
        x1 = np.empty_like(x1p)
        x1[self.perm] = x1p
        X = np.vstack([x1, x2])
        return X[:, 0] if one else X

    def inv_diag(self, idx, chunk: int = 64):
        """(Q^{-1})_{kk} for k in idx, one unit-vector solve per index."""
        idx = np.asarray(idx, np.int64)
        out = np.empty(idx.shape[0])
        for c0 in range(0, idx.shape[0], chunk):
            ks = idx[c0:c0 + chunk]
            E = np.zeros((self.N, ks.shape[0]))
            E[ks, np.arange(ks.shape[0])] = 1.0
            X = self.solve(E)
            out[c0:c0 + chunk] = X[ks, np.arange(ks.shape[0])]
        return out


def factor(Q, a: int, method: str = "auto"):
    N = Q.shape[0]
    if method == "auto":
        method = "dense" if N <= 6000 else "banded"
    if method == "dense":
        return DenseSPD(Q)
    return BandedSPD(Q, a)
