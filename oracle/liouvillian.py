"""Explicit HEOM Liouvillian superoperator (HEOMLS) -- oracle (test
infrastructure only).

Assembles the matrix M of eq:HEOM by Kronecker products, term by term,
in the paper's notation:

  d/dt rho_{j|q} = -(i L_s + sum_r chi_{j_r} + sum_w gamma_{q_w}) rho_{j|q}
                   - i sum_{q' not in q} A_{q'} rho_{j|q+}
                   - i sum_{j'}          B_{j'} rho_{j+|q}
                   - i sum_w (-1)^(n-w)  C_{q_w} rho_{j|q_w^-}
                   - i sum_r             D_{j_r} rho_{j_r^-|q}

with (the superoperator definitions right after eq:HEOM)
  A_q[.] = (-1)^{delta_{p,-}} { d^{nubar} [.] - P_s[[.] d^{nubar}] }
  C_q[.] = (-1)^{delta_{p,-}} { eta^nu d^nu [.] + (eta^{nubar})^* P_s[[.] d^nu] }
  B_j[.] = [V, .]
  D_j[.] = delta_{u,R} xi^R [V, .] + i delta_{u,I} xi^I {V, .}
  P_s[rho^{(m,n,+-)} d] = -+ (-1)^n rho^{(m,n,+-)} d.

Readings: the level n inside P_s is that of the ADO the superoperator
acts on; d^{+1} = d^dagger, d^{-1} = d; an "RI" bosonic exponent (real
chi) carries both parts, D = Re(xi)[V,.] + i Im(xi){V,.}; fermionic ADOs
are antisymmetric (see hierarchy.py), so rho_{[q', q_n..q_1]} equals the
permutation sign times the stored ADO.

Vectorisation is column stacking, vec(A X B) = (B^T kron A) vec(X), so
spre(A) = I kron A and spost(B) = B^T kron I.  ``rowmajor_permutation``
converts to the GPU library's row-major [N][d][d] layout.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .hierarchy import OracleHierarchy, ferm_importance_rank, importance_value


# ---------------------------------------------------------------------------
# Model description: the paper's inputs (Fig. 1a-b): H_s, coupling operators
# and exponent lists, flattened into one exponent list per statistics.
# ---------------------------------------------------------------------------
def flatten_baths(baths):
    """Bath records -> (bosonic exponent list, fermionic exponent list).

    Bosonic record: dict(kind="boson", op=V, u_type=[...], xi=[...], chi=[...])
      u_type in {"R", "I", "RI"}; one exponent per entry, in record order.
    Fermionic record: dict(kind="fermion", op=d (annihilation),
      eta_p, gam_p, eta_m, gam_m) -- h-paired lists for nu = +1 and -1.
      Exponent order: for h = 0..: nu = +1 then nu = -1.
    """
    bos, ferm = [], []
    for rec in baths:
        op = np.asarray(rec["op"], dtype=np.complex128)
        if rec["kind"] == "boson":
            for u, xi, chi in zip(rec["u_type"], rec["xi"], rec["chi"]):
                bos.append(dict(op=op, u=u, xi=complex(xi), chi=complex(chi)))
        else:
            base = len(ferm)
            n = len(rec["eta_p"])
            for h in range(n):
                ferm.append(dict(op=op, nu=+1, eta=complex(rec["eta_p"][h]), gamma=complex(rec["gam_p"][h]),
                                 partner=base + 2 * h + 1))
                ferm.append(dict(op=op, nu=-1, eta=complex(rec["eta_m"][h]), gamma=complex(rec["gam_m"][h]),
                                 partner=base + 2 * h))
    return bos, ferm


def _dnu(op, nu):
    """d^nu: nu = +1 -> d^dagger, nu = -1 -> d."""
    return op.conj().T if nu == +1 else op


def spre(A):
    d = A.shape[0]
    return sp.kron(sp.identity(d, format="csr"), sp.csr_matrix(A), format="csr")


def spost(B):
    d = B.shape[0]
    return sp.kron(sp.csr_matrix(B.T), sp.identity(d, format="csr"), format="csr")


def _ps_factor(parity: int, n_acted: int) -> int:
    """P_s[rho^{(m,n,p)} d] = -p (-1)^n rho d  (p = +1 or -1)."""
    return -parity * (-1) ** n_acted


def _pf(parity: int) -> int:
    """(-1)^{delta_{p,-}}."""
    return 1 if parity == +1 else -1


class OracleHEOM:
    """Sparse HEOMLS for given H, baths, truncation and parity."""

    def __init__(self, H, baths, m_max, n_max, parity=+1, ferm_perm=None, importance_threshold=0.0, lindblad=()):
        """ferm_perm: optional relabelling of the fermionic exponents (new
        position i holds old exponent ferm_perm[i]); used to check that
        physical results do not depend on the exponent order.
        importance_threshold > 0: leave out the ADOs of eq:importance below
        it (levels m > 1 or n > 1); terms that reach a left-out ADO are
        dropped like those beyond the tier cutoff.
        lindblad: jump operators F; every ADO gets the Lindbladian of
        eq:Lindbladian, F [.] F^dagger - 1/2 {F^dagger F, .}, beside its own
        terms (the ADO space does not grow)."""
        self.H = np.asarray(H, dtype=np.complex128)
        self.lindblad = [np.asarray(F, dtype=np.complex128) for F in lindblad]
        self.d = self.H.shape[0]
        self.bos, self.ferm = flatten_baths(baths)
        self.ferm_rank = ferm_importance_rank([len(r["eta_p"]) for r in baths if r["kind"] != "boson"])
        if ferm_perm is not None:
            inv = {old: new for new, old in enumerate(ferm_perm)}
            self.ferm = [dict(self.ferm[old], partner=inv[self.ferm[old]["partner"]]) for old in ferm_perm]
        self.parity = parity
        imp = None
        if importance_threshold > 0:
            if ferm_perm is not None:
                raise ValueError("importance pruning with a relabelled exponent list is not defined")
            imp = lambda j, q: importance_value(j, q, self.bos, self.ferm, self.ferm_rank)
        self.hier = OracleHierarchy(len(self.bos), m_max, len(self.ferm), n_max, importance=imp,
                                    threshold=importance_threshold)
        self.N = len(self.hier)
        self._cache = {}

    # -- superoperator pieces -------------------------------------------------
    def _pre(self, key, A):
        k = ("pre", key)
        if k not in self._cache:
            self._cache[k] = spre(A).tocoo()
        return self._cache[k]

    def _post(self, key, B):
        k = ("post", key)
        if k not in self._cache:
            self._cache[k] = spost(B).tocoo()
        return self._cache[k]

    def _terms_A(self, qp, n_acted):
        """A_{q'} as (coefficient, superop) pairs."""
        e = self.ferm[qp]
        dn = _dnu(e["op"], -e["nu"])
        key = ("f", qp, -e["nu"])
        pf = _pf(self.parity)
        return [(pf, self._pre(key, dn)), (-pf * _ps_factor(self.parity, n_acted), self._post(key, dn))]

    def _terms_C(self, q, n_acted):
        e = self.ferm[q]
        dn = _dnu(e["op"], e["nu"])
        key = ("f", q, e["nu"])
        pf = _pf(self.parity)
        eta = e["eta"]
        etabar = self.ferm[e["partner"]]["eta"]
        return [(pf * eta, self._pre(key, dn)),
                (pf * np.conj(etabar) * _ps_factor(self.parity, n_acted), self._post(key, dn))]

    def _terms_B(self, j):
        V = self.bos[j]["op"]
        key = ("b", j)
        return [(1.0, self._pre(key, V)), (-1.0, self._post(key, V))]

    def _terms_D(self, j):
        e = self.bos[j]
        V = e["op"]
        key = ("b", j)
        if e["u"] == "R":
            xr, xi = e["xi"], 0.0
        elif e["u"] == "I":
            xr, xi = 0.0, e["xi"]
        else:  # combined real/imaginary exponent with real chi
            xr, xi = e["xi"].real, e["xi"].imag
        # xr [V, .] + i xi {V, .}
        return [(xr + 1j * xi, self._pre(key, V)), (-xr + 1j * xi, self._post(key, V))]

    # -- assembly ------------------------------------------------------------------
    def block_terms(self, a):
        """All (column ADO, coefficient, superop) contributions to block row a."""
        hier = self.hier
        j, q = hier.ados[a]
        m, n = len(j), len(q)
        out = []
        Hk = ("H",)
        decay = sum(self.bos[x]["chi"] for x in j) + sum(self.ferm[x]["gamma"] for x in q)
        # -(i L_s + decay) rho
        out.append((a, -1j, self._pre(Hk, self.H)))
        out.append((a, 1j, self._post(Hk, self.H)))
        out.append((a, -decay, None))
        # eq:Lindbladian for every jump operator F
        for k, F in enumerate(self.lindblad):
            Fd = F.conj().T
            key = ("L", k)
            if key not in self._cache:
                self._cache[key] = (spre(F) @ spost(Fd)).tocoo()
            out.append((a, 1.0, self._cache[key]))
            out.append((a, -0.5, self._pre(("LL", k), Fd @ F)))
            out.append((a, -0.5, self._post(("LL", k), Fd @ F)))
        # -i sum_{q' not in q} A_{q'} rho_{j|[q', q]}
        if n < hier.Lf:
            for qp in range(len(self.ferm)):
                if qp in q:
                    continue
                b, sgn = hier.lookup(j, (qp,) + q)
                if b is None:
                    continue
                for c, S in self._terms_A(qp, n + 1):
                    out.append((b, -1j * sgn * c, S))
        # -i sum_{j'} B_{j'} rho_{j+|q}
        if m < hier.Lb:
            for jp in range(len(self.bos)):
                b, _ = hier.lookup((jp,) + j, q)
                if b is None:
                    continue
                for c, S in self._terms_B(jp):
                    out.append((b, -1j * c, S))
        # -i sum_{w=1}^{n} (-1)^(n-w) C_{q_w} rho_{j|q_w^-};  q = [q_n .. q_1]
        for w in range(1, n + 1):
            pos = n - w                      # list position of q_w
            qw = q[pos]
            rest = q[:pos] + q[pos + 1:]
            b, sgn = hier.lookup(j, rest)
            if b is None:            # left out by the importance threshold
                continue
            assert sgn == 1
            for c, S in self._terms_C(qw, n - 1):
                out.append((b, -1j * (-1) ** (n - w) * c, S))
        # -i sum_{r=1}^{m} D_{j_r} rho_{j_r^-|q}
        for r in range(m):
            jr = j[r]
            rest = j[:r] + j[r + 1:]
            b, _ = hier.lookup(rest, q)
            if b is None:            # left out by the importance threshold
                continue
            for c, S in self._terms_D(jr):
                out.append((b, -1j * c, S))
        return out

    def drive_superop(self, V):
        """-i[V, .] on every ADO (block diagonal): the part of the first line
        of eq:HEOM that a term f(t) V of a time-dependent H_s(t) adds."""
        V = np.asarray(V, dtype=np.complex128)
        blk = (-1j * (spre(V) - spost(V))).tocsr()
        return sp.kron(sp.identity(self.N, format="csr"), blk, format="csr")

    def assemble(self, rows=None, shift=0.0):
        """CSR matrix of M + shift*I (column-stacked blocks, oracle order).

        rows: optional list of block rows; then the result has
        len(rows)*d^2 rows (in the given order) and N*d^2 columns."""
        d2 = self.d * self.d
        rows = range(self.N) if rows is None else list(rows)
        R, C, V = [], [], []
        eye = np.arange(d2)
        for out_i, a in enumerate(rows):
            r0 = out_i * d2
            for b, coef, S in self.block_terms(a):
                if S is None:
                    R.append(r0 + eye)
                    C.append(b * d2 + eye)
                    V.append(np.full(d2, coef + shift, dtype=np.complex128))
                    continue
                if coef == 0:
                    continue
                R.append(r0 + S.row)
                C.append(b * d2 + S.col)
                V.append(coef * S.data)
        Mx = sp.coo_matrix((np.concatenate(V), (np.concatenate(R), np.concatenate(C))),
                           shape=(len(rows) * d2, self.N * d2)).tocsr()
        Mx.sum_duplicates()
        return Mx


def rowmajor_permutation(N, d):
    """Index array P with v_rowmajor = v_colstack[P] for [N][d][d] blocks."""
    a = np.arange(N)[:, None, None]
    i = np.arange(d)[None, :, None]
    j = np.arange(d)[None, None, :]
    return (a * d * d + i + j * d).reshape(-1)


def to_blocks(v_colstack, N, d):
    """Column-stacked vector -> array [N][d][d] (row-major blocks)."""
    return np.asarray(v_colstack)[rowmajor_permutation(N, d)].reshape(N, d, d)


def from_blocks(x):
    """Array [N][d][d] -> column-stacked vector."""
    x = np.asarray(x)
    return np.transpose(x, (0, 2, 1)).reshape(-1)
