"""Solvers on the assembled HEOMLS -- oracle (test infrastructure only).

* ``rk4``: classical fourth-order Runge-Kutta on dx/dt = M x (the paper
  integrates eq:HEOM with an adaptive ODE solver; fixed-step RK4 is the
  method the GPU library implements, so both sides take the same steps).
* ``steady_state``: the stationary ADOs, M x = 0 with the normalisation
  Tr rho_0 = 1.  Reading: the paper only says a linear solver is used; the
  equation for element (0,0) of the reduced density operator (ADO 0) is
  replaced by the trace condition, which is consistent because the trace
  of the ADO-0 block of M x vanishes for every x in the even sector.
* ``dos`` and ``psd``: Methods, "Numerical computation of the spectrum":
    pi S(w) = -Re Tr[a^dag x],  (M - i w) x = a rho_ss         (even M)
    pi A(w) = -Re{Tr[d x_+] + Tr[d^dag x_-]},
        (M + i w) x_+ = d^dag rho_ss, (M - i w) x_- = d rho_ss  (odd M)
  where the right-hand side left-multiplies every ADO of the stationary
  state and only the reduced density operator (ADO 0) of x is traced.
All vectors here are column-stacked (see liouvillian.py).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .liouvillian import from_blocks, to_blocks


def rk4(M, x0, dt, n_steps, save_every=0, d=None):
    """Fixed-step RK4; returns final x and (optionally) the reduced density
    operator every save_every steps (d must then be given)."""
    x = np.array(x0, dtype=np.complex128)
    traj = []
    for s in range(n_steps):
        k1 = M @ x
        k2 = M @ (x + 0.5 * dt * k1)
        k3 = M @ (x + 0.5 * dt * k2)
        k4 = M @ (x + dt * k3)
        x = x + (dt / 6.0) * (k1 + 2 * k2 + 2 * k3 + k4)
        if save_every and (s + 1) % save_every == 0:
            traj.append(x[: d * d].reshape(d, d, order="F").copy())
    return x, traj


def rk4_driven(M0, drives, f, x0, t0, dt, n_steps):
    """RK4 on dx/dt = M(t) x with a time-dependent system Hamiltonian
    H_s(t) = H + sum_k f_k(t) V_k (the paper allows H_s(t) in the dynamics):
    M(t) = M0 + sum_k f_k(t) D_k with D_k = -i[V_k, .] on every ADO (see
    OracleHEOM.drive_superop).  f(t) returns the real coefficients f_k(t);
    the stages use the times t, t + dt/2, t + dt/2, t + dt."""
    x = np.array(x0, dtype=np.complex128)

    def M(t):
        c = f(t)
        return M0 + sum(ck * Dk for ck, Dk in zip(c, drives))

    t = t0
    for _ in range(n_steps):
        Ma, Mb, Mc = M(t), M(t + 0.5 * dt), M(t + dt)
        k1 = Ma @ x
        k2 = Mb @ (x + 0.5 * dt * k1)
        k3 = Mb @ (x + 0.5 * dt * k2)
        k4 = Mc @ (x + dt * k3)
        x = x + (dt / 6.0) * (k1 + 2 * k2 + 2 * k3 + k4)
        t += dt
    return x


def bordered_matrix(M, d):
    """Replace the row of element (0,0) of ADO 0 by the trace row."""
    M = sp.csr_matrix(M, dtype=np.complex128, copy=True)
    M.data[M.indptr[0]:M.indptr[1]] = 0.0   # drop row 0
    M.eliminate_zeros()
    cols = [i + i * d for i in range(d)]    # column-stacked index of rho_0[i, i]
    trace_row = sp.csr_matrix((np.ones(d, dtype=np.complex128), ([0] * d, cols)), shape=M.shape)
    return (M + trace_row).tocsc()


def _splu_solve(A, b):
    return spla.splu(sp.csc_matrix(A)).solve(b)


def steady_state(M, d, solve=None):
    """Stationary state: B x = e_0 with the bordered matrix B.  solve(A, b)
    is the linear solver, sparse LU by default."""
    B = bordered_matrix(M, d)
    b = np.zeros(M.shape[0], dtype=np.complex128)
    b[0] = 1.0
    return (solve or _splu_solve)(B, b)


def left_multiply_all(x, op, N, d):
    """b = (I kron O) x blockwise: O @ rho_a for every ADO a."""
    blocks = to_blocks(x, N, d)
    return from_blocks(np.einsum("ik,akj->aij", op, blocks))


def dos(M_odd, x_ss, dop, omegas, N, d, solve=None):
    """Density of states A(w) of the fermionic operator d (odd-parity M).
    solve(A, b) is the linear solver, sparse LU by default."""
    solve = solve or _splu_solve
    dd = dop.conj().T
    b_plus = left_multiply_all(x_ss, dd, N, d)
    b_minus = left_multiply_all(x_ss, dop, N, d)
    I = sp.identity(M_odd.shape[0], format="csc", dtype=np.complex128)
    out = []
    for w in omegas:
        xp = solve(M_odd + 1j * w * I, b_plus)
        xm = solve(M_odd - 1j * w * I, b_minus)
        r0p = xp[: d * d].reshape(d, d, order="F")
        r0m = xm[: d * d].reshape(d, d, order="F")
        out.append(-(np.trace(dop @ r0p) + np.trace(dd @ r0m)).real / np.pi)
    return np.array(out)


def psd(M_even, x_ss, aop, omegas, N, d, solve=None):
    """Power spectral density S(w) of the bosonic operator a (even M).
    solve(A, b) is the linear solver, sparse LU by default."""
    solve = solve or _splu_solve
    b = left_multiply_all(x_ss, aop, N, d)
    I = sp.identity(M_even.shape[0], format="csc", dtype=np.complex128)
    out = []
    for w in omegas:
        x = solve(M_even - 1j * w * I, b)
        r0 = x[: d * d].reshape(d, d, order="F")
        out.append(-(np.trace(aop.conj().T @ r0)).real / np.pi)
    return np.array(out)


def gmres_jacobi(A, b, tol=1e-8, restart=30, maxiter=2000):
    """scipy GMRES with a Jacobi (diagonal) preconditioner; used only to time
    an iterative CPU solve beside the GPU one."""
    dg = A.diagonal().copy()
    dg[np.abs(dg) < 1e-300] = 1.0
    Pinv = spla.LinearOperator(A.shape, matvec=lambda v: v / dg, dtype=np.complex128)
    it = [0]

    def cb(_):
        it[0] += 1

    x, info = spla.gmres(A, b, rtol=tol, restart=restart, maxiter=maxiter, M=Pinv, callback=cb,
                         callback_type="pr_norm")
    return x, info, it[0]


class _OutOfTime(Exception):
    pass


def gmres_jacobi_timed(A, b, tol=1e-10, mark=1e-8, restart=30, maxiter=100000, max_seconds=None):
    """gmres_jacobi with a clock: the returned record holds the iteration and
    the elapsed seconds at which the relative preconditioned residual first
    fell to `mark`, and the total.  With max_seconds the solve stops once
    that much time has passed (x is then None): a bounded sample of the
    iteration cost."""
    import time
    dg = A.diagonal().copy()
    dg[np.abs(dg) < 1e-300] = 1.0
    Pinv = spla.LinearOperator(A.shape, matvec=lambda v: v / dg, dtype=np.complex128)
    rec = {"iterations": 0, "mark": mark, "mark_iteration": None, "mark_seconds": None, "last_residual": None}
    t0 = time.perf_counter()

    def cb(r):
        rec["iterations"] += 1
        rec["last_residual"] = float(r)
        el = time.perf_counter() - t0
        if rec["mark_iteration"] is None and r <= mark:
            rec["mark_iteration"], rec["mark_seconds"] = rec["iterations"], el
        if max_seconds is not None and el > max_seconds:
            raise _OutOfTime

    x, info = None, None
    try:
        x, info = spla.gmres(A, b, rtol=tol, restart=restart, maxiter=maxiter, M=Pinv, callback=cb,
                             callback_type="pr_norm")
    except _OutOfTime:
        pass
    rec["seconds"] = time.perf_counter() - t0
    rec["info"] = info
    return x, rec
