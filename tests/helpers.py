"""Shared test plumbing: build the oracle and the library on the same inputs
and map between their ADO orders.  Holds no HEOM arithmetic."""
import numpy as np

from oracle import exponents as ox
from oracle.liouvillian import OracleHEOM, from_blocks, to_blocks


def oracle_model(cfg, parity=+1, m_max=None, n_max=None, baths=None):
    b = ox.exponent_records(baths if baths is not None else cfg["baths"])
    return OracleHEOM(cfg["H"], b, cfg.get("m_max", 0) if m_max is None else m_max,
                      cfg.get("n_max", 0) if n_max is None else n_max, parity=parity)


def library_model(cfg, parity=+1, m_max=None, n_max=None, baths=None, parity_op=None):
    from paper_2306_07522_amd import api
    return api.Hierarchy(cfg["H"], baths if baths is not None else cfg["baths"],
                         cfg.get("m_max", 0) if m_max is None else m_max,
                         cfg.get("n_max", 0) if n_max is None else n_max, parity=parity, parity_op=parity_op)


def oracle_to_library_perm(om, lm):
    """perm[k] = library index of the oracle's ADO k (same stored sign
    convention on both sides, so no sign)."""
    occ, mask, _ = lm.ados()
    key = {}
    for a in range(lm.N):
        key[(tuple(int(v) for v in occ[a]), int(mask[a]))] = a
    perm = np.empty(om.N, dtype=np.int64)
    Kb = lm.Kb
    for k, (j, q) in enumerate(om.hier.ados):
        o = [0] * Kb
        for x in j:
            o[x] += 1
        m = 0
        for x in q:
            m |= 1 << x
        perm[k] = key[(tuple(o), m)]
    return perm


def rel_err(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) / max(np.linalg.norm(np.asarray(b).ravel()), 1e-300))
