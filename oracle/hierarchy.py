"""ADO enumeration and hierarchy dictionary -- oracle (test infrastructure only).

An ADO rho^{(m,n,p)}_{j|q} (Results, the paragraph introducing ADOs and
eq:HEOM) is labelled by a bosonic vector j = [j_m..j_1] and a fermionic
vector q = [q_n..q_1] of exponent indices.  Truncation: m <= m_max,
n <= n_max (the paragraph after the P_s definition); q' not in q (Pauli).

Readings:
* bosonic ADOs are symmetric in j: one ADO per multiset, stored as the
  ascending tuple of exponent indices (so j_r with repeats appear);
* fermionic ADOs are antisymmetric in q: one ADO per set, stored as the
  descending tuple (q_n > ... > q_1) of exponent indices (Table 3's
  counts are binomials, one ADO per set).

The enumeration is itertools over multisets and subsets, ordered by
bosonic multiset first, then fermionic subset -- an order chosen for
simplicity, unrelated to the GPU library's.
"""
from __future__ import annotations

import itertools


class OracleHierarchy:
    def __init__(self, n_bos_exp: int, m_max: int, n_ferm_exp: int, n_max: int, importance=None, threshold=0.0):
        """importance: optional callable (j, q) -> importance value of the ADO
        (see ``importance_value``); with threshold > 0, ADOs with m > 1 or
        n > 1 whose importance is below the threshold are left out (the
        truncation paragraph after eq:HEOM, eq:importance)."""
        self.Kb, self.Lb, self.Kf, self.Lf = n_bos_exp, m_max, n_ferm_exp, n_max
        bos = [()]
        if self.Kb > 0:
            for m in range(1, self.Lb + 1):
                bos.extend(itertools.combinations_with_replacement(range(self.Kb), m))
        ferm = [()]
        for n in range(1, min(self.Lf, self.Kf) + 1):
            ferm.extend(tuple(sorted(c, reverse=True)) for c in itertools.combinations(range(self.Kf), n))
        self.ados = [(j, q) for j in bos for q in ferm]
        if importance is not None and threshold > 0:
            self.ados = [(j, q) for j, q in self.ados
                         if (len(j) <= 1 and len(q) <= 1) or importance(j, q) >= threshold]
        self.index = {key: i for i, key in enumerate(self.ados)}

    def __len__(self):
        return len(self.ados)

    def lookup(self, j, q):
        """Index of the ADO with bosonic multiset j and fermionic set q,
        with the sign that turns the given ordered fermionic vector into the
        stored (descending) one: rho_{[q as given]} = sign * rho_stored.
        Returns (index, sign) or (None, 0) if truncated away."""
        jj = tuple(sorted(j))
        qq = list(q)
        if len(set(qq)) != len(qq):
            return None, 0
        sign = permutation_sign_to_descending(qq)
        key = (jj, tuple(sorted(qq, reverse=True)))
        idx = self.index.get(key)
        if idx is None:
            return None, 0
        return idx, sign


def importance_value(j, q, bos, ferm, ferm_rank):
    """eq:importance: |prod_r xi_{j_r} / (Re chi_{j_r} sum_{x<=r} Re chi_{j_x})|
    times |prod_w eta_{q_w} / (Re gamma_{q_w} sum_{x<=w} Re gamma_{q_x})|.

    Reading of the order the products and partial sums run in: ascending
    position in the exponent list, the bosonic list in record order and the
    fermionic list ordered by ``ferm_rank`` -- each fermionic bath's nu = +1
    terms h = 1..N_alpha, then its nu = -1 terms.  With that order the counts
    of Table 3 (example 1, 56 exponents) are reproduced; ordering by decay
    rate or with nu interleaved per h does not reproduce them.
    bos / ferm: lists of dicts with 'xi', 'chi' / 'eta', 'gamma'."""
    value = 1.0
    s = 0.0
    for x in sorted(j):
        rc = bos[x]["chi"].real
        s += rc
        value *= abs(bos[x]["xi"]) / rc / s
    s = 0.0
    for x in sorted(q, key=lambda k: ferm_rank[k]):
        rg = ferm[x]["gamma"].real
        s += rg
        value *= abs(ferm[x]["eta"]) / rg / s
    return value


def ferm_importance_rank(n_terms_per_bath):
    """Rank of every fermionic exponent in the flattened (h, nu = +1 / -1)
    interleaved list: per bath, its nu = +1 terms first, then nu = -1."""
    rank, base = [], 0
    for n in n_terms_per_bath:
        for h in range(n):
            rank.append(base + h)          # nu = +1, term h
            rank.append(base + n + h)      # nu = -1, term h
        base += 2 * n
    return rank


def permutation_sign_to_descending(seq) -> int:
    """Sign of the permutation that sorts seq into descending order,
    computed by counting bubble-sort transpositions."""
    a = list(seq)
    sign = 1
    n = len(a)
    for i in range(n):
        for k in range(n - 1 - i):
            if a[k] < a[k + 1]:
                a[k], a[k + 1] = a[k + 1], a[k]
                sign = -sign
    return sign
