"""Python binding of the HEOM library: argument marshalling only.

Every computation happens inside libheom.so (host setup in C++, every step
of the hot path in HIP kernels); this module converts numpy arrays and torch
tensors to the pointers and sizes of the C ABI (include/heom.h).  Device
vectors are torch tensors (complex128 for FP64, complex64 for FP32) on the
current HIP device; streams are torch's current stream unless given.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as L


def _dptr(a):
    return a.ctypes.data_as(L.dp)


def _c128(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.complex128))


def lib():
    return L.load()


# ----------------------------------------------------------------- exponents
def pade_params(kind: str, n: int, method: str = "pade"):
    lb = lib()
    k = np.zeros(max(n, 1))
    z = np.zeros(max(n, 1))
    L.check(lb.heom_pade_params(L.HEOM_FERMION if kind == "fermi" else L.HEOM_BOSON,
                                L.HEOM_PADE if method == "pade" else L.HEOM_MATSUBARA, n, _dptr(k), _dptr(z)))
    return k[:n], z[:n]


def exponents_lorentz(Gamma, W, mu, T, n_exp, method="pade"):
    lb = lib()
    out = [np.zeros(n_exp, dtype=np.complex128) for _ in range(4)]
    L.check(lb.heom_exponents_lorentz(Gamma, W, mu, T, n_exp, L.HEOM_PADE if method == "pade" else L.HEOM_MATSUBARA,
                                      *[_dptr(o) for o in out]))
    return dict(eta_p=out[0], gam_p=out[1], eta_m=out[2], gam_m=out[3])


def exponents_drude_lorentz(lam, gamma, T, n_exp, method="matsubara"):
    lb = lib()
    xi = np.zeros(n_exp, dtype=np.complex128)
    chi = np.zeros(n_exp, dtype=np.complex128)
    L.check(lb.heom_exponents_drude_lorentz(lam, gamma, T, n_exp,
                                            L.HEOM_PADE if method == "pade" else L.HEOM_MATSUBARA,
                                            _dptr(xi), _dptr(chi)))
    return xi, chi


_UTYPE = {"R": L.HEOM_U_R, "I": L.HEOM_U_I, "RI": L.HEOM_U_RI}


def _bath_struct(rec, keep):
    """One bath record (physical spectral parameters or raw exponents) ->
    heom_bath; arrays are appended to `keep` to outlive the call."""
    b = L.heom_bath()
    op = _c128(rec["op"])
    keep.append(op)
    b.op = _dptr(op)
    if rec["kind"] == "boson":
        b.kind = L.HEOM_BOSON
        if rec.get("spectral") == "drude_lorentz":
            xi, chi = exponents_drude_lorentz(rec["lam"], rec["gamma"], rec["T"], rec["n_exp"],
                                              rec.get("method", "matsubara"))
            ut = np.full(len(xi), L.HEOM_U_RI, dtype=np.int32)
        else:
            xi, chi = _c128(rec["xi"]), _c128(rec["chi"])
            ut = np.array([_UTYPE[u] for u in rec["u_type"]], dtype=np.int32)
        keep += [xi, chi, ut]
        b.n_exp = len(xi)
        b.u_type = ut.ctypes.data_as(L.i32p)
        b.xi = _dptr(xi)
        b.chi = _dptr(chi)
    else:
        b.kind = L.HEOM_FERMION
        if rec.get("spectral") == "lorentz":
            e = exponents_lorentz(rec["Gamma"], rec["W"], rec["mu"], rec["T"], rec["n_exp"], rec.get("method", "pade"))
        else:
            e = {k: _c128(rec[k]) for k in ("eta_p", "gam_p", "eta_m", "gam_m")}
        keep += list(e.values())
        b.n_exp = len(e["eta_p"])
        b.eta_p, b.gam_p, b.eta_m, b.gam_m = (_dptr(e[k]) for k in ("eta_p", "gam_p", "eta_m", "gam_m"))
    return b


def _stream_ptr(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _precision_of(t):
    import torch
    if t.dtype == torch.complex128:
        return L.HEOM_FP64
    if t.dtype == torch.complex64:
        return L.HEOM_FP32
    raise TypeError(f"ADO vectors must be complex128 or complex64 tensors, got {t.dtype}")


def _devptr(t):
    if not t.is_cuda:
        raise ValueError("device vectors must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("device vectors must be contiguous")
    return C.c_void_p(t.data_ptr())


class Hierarchy:
    """Handle of heom_build_hierarchy: ADO list, neighbour tables, operators."""

    def __init__(self, H, baths, m_max, n_max, parity=+1, parity_op=None, importance_threshold=0.0, lindblad=()):
        lb = lib()
        H = _c128(H)
        d = H.shape[0]
        keep = []
        structs = (L.heom_bath * max(len(baths), 1))()
        for i, rec in enumerate(baths):
            structs[i] = _bath_struct(rec, keep)
        pop = None
        if parity_op is not None:
            pop = _c128(parity_op)
        h = C.c_void_p()
        if importance_threshold > 0:
            L.check(lb.heom_build_hierarchy_pruned(d, _dptr(H), len(baths), structs, m_max, n_max, parity,
                                                   _dptr(pop) if pop is not None else None,
                                                   float(importance_threshold), C.byref(h)))
        else:
            L.check(lb.heom_build_hierarchy(d, _dptr(H), len(baths), structs, m_max, n_max, parity,
                                            _dptr(pop) if pop is not None else None, C.byref(h)))
        self._h = h
        self._lib = lb
        info = L.heom_info()
        L.check(lb.heom_hierarchy_info(h, C.byref(info)))
        self.info = info
        self.N = info.n_ado
        self.d = info.d
        self.Kb = info.n_bos_exp
        self.Kf = info.n_ferm_exp
        self.parity = parity
        if len(lindblad):
            self.set_lindblad(lindblad)

    def set_lindblad(self, ops):
        """Jump operators F_k (eq:Lindbladian): every ADO also evolves under
        sum_k F_k X F_k^dagger - 1/2 {F_k^dagger F_k, X}; rates go into F_k."""
        ops = [_c128(F) for F in ops]
        if ops:
            arr = np.ascontiguousarray(np.stack(ops)).view(np.float64)
            L.check(self._lib.heom_hierarchy_set_lindblad(self._h, len(ops), arr.ctypes.data_as(L.dp)))
        else:
            L.check(self._lib.heom_hierarchy_set_lindblad(self._h, 0, None))

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            self._lib.heom_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def tier_offsets(self):
        return [self.info.tier_offset[t] for t in range(self.info.n_tiers + 1)]

    def ados(self):
        """(bos_occ [N][K_b], ferm_mask [N], level [N][2])."""
        occ = np.zeros((self.N, max(self.Kb, 1)), dtype=np.int32)
        mask = np.zeros(self.N, dtype=np.uint64)
        lev = np.zeros((self.N, 2), dtype=np.int32)
        L.check(self._lib.heom_hierarchy_ados(self._h, occ.ctypes.data_as(L.i32p), mask.ctypes.data_as(L.u64p),
                                              lev.ctypes.data_as(L.i32p)))
        return occ[:, : self.Kb], mask, lev

    def index(self, bos_occ, ferm_ids):
        occ = np.ascontiguousarray(np.asarray(bos_occ if len(bos_occ) else [0], dtype=np.int32))
        ids = np.ascontiguousarray(np.asarray(ferm_ids if len(ferm_ids) else [0], dtype=np.int32))
        idx = C.c_int64()
        sgn = C.c_int32()
        L.check(self._lib.heom_ado_index(self._h, occ.ctypes.data_as(L.i32p), ids.ctypes.data_as(L.i32p),
                                         len(ferm_ids), C.byref(idx), C.byref(sgn)))
        return idx.value, sgn.value

    def tables(self):
        E = self.info.n_edges
        dec = np.zeros(self.N, dtype=np.complex128)
        rp = np.zeros(self.N + 1, dtype=np.int64)
        col, kind, expo, mult = (np.zeros(max(E, 1), dtype=np.int32) for _ in range(4))
        L.check(self._lib.heom_hierarchy_tables(self._h, _dptr(dec), rp.ctypes.data_as(L.i64p),
                                                *[a.ctypes.data_as(L.i32p) for a in (col, kind, expo, mult)]))
        return dict(decay=dec, row_ptr=rp, col=col[:E], kind=kind[:E], exp=expo[:E], mult=mult[:E])

    def slab_plan_stats(self):
        """Host-side layout of the slab launch plan (heom_slab_plan_stats), or
        None when the hierarchy has no slab plan."""
        st = L.heom_slab_stats()
        L.check(self._lib.heom_slab_plan_stats(self._h, C.byref(st)))
        if not st.built:
            return None
        return dict(children=st.children, parents=st.parents, jobs=list(st.jobs), entries=list(st.entries),
                    max_vertices=list(st.max_vertices), cost=list(st.cost),
                    xcd_cost=[list(st.xcd_cost[l]) for l in range(2)])

    # ------------------------------------------------------------ device work
    def prepare(self):
        """Upload the device tables now (heom_prepare)."""
        L.check(self._lib.heom_prepare(self._h))

    def apply(self, x, y=None, shift=None, n_rhs=1, stream=None, tiled=None, plan=None):
        """y = (M + shift) x on the GPU.  x: [N][d][d] or [N][d][d][R] tensor.
        shift: complex scalar, or a device tensor of R shifts (per column).
        plan: None (library default), "pull", "slab" or "pull_mfma" (heom_apply_plan)."""
        import torch
        if y is None:
            y = torch.empty_like(x)
        prec = _precision_of(x)
        if y.dtype != x.dtype:
            raise TypeError("x and y must have the same dtype")
        if x.numel() != self.N * self.d * self.d * n_rhs:
            raise ValueError("x has the wrong size for this hierarchy")
        s = _stream_ptr(stream)
        if isinstance(shift, torch.Tensor):
            if shift.dtype != x.dtype or shift.numel() != n_rhs:
                raise ValueError("per-RHS shifts: one complex of the vector dtype per column")
            L.check(self._lib.heom_apply_shifted(self._h, prec, _devptr(x), _devptr(y), n_rhs, _devptr(shift), s))
            return y
        sh = None
        if shift is not None:
            sh = np.array([complex(shift).real, complex(shift).imag])
        if plan is not None:
            code = {"auto": 0, "pull": 1, "slab": 2, "pull_mfma": 3}[plan]
            L.check(self._lib.heom_apply_plan(self._h, prec, _devptr(x), _devptr(y), n_rhs,
                                              _dptr(sh) if sh is not None else None, code, s))
        elif tiled is not None:
            L.check(self._lib.heom_apply_tiled(self._h, prec, _devptr(x), _devptr(y), n_rhs,
                                               _dptr(sh) if sh is not None else None, int(tiled), s))
        else:
            L.check(self._lib.heom_apply(self._h, prec, _devptr(x), _devptr(y), n_rhs,
                                         _dptr(sh) if sh is not None else None, s))
        return y


def apply_steady_operator(h, x, y=None, stream=None):
    """y = B x, the bordered stationary-state operator (see heom.h)."""
    import torch
    if y is None:
        y = torch.empty_like(x)
    L.check(lib().heom_apply_steady_operator(h.handle, _precision_of(x), _devptr(x), _devptr(y), _stream_ptr(stream)))
    return y


# ----------------------------------------------------------------- solvers
_PREC = {"none": L.HEOM_PREC_NONE, "jacobi": L.HEOM_PREC_JACOBI, "nn": L.HEOM_PREC_NN, "scaled": L.HEOM_PREC_SCALED,
         "block": L.HEOM_PREC_BLOCK}
_MODE = {"fp64": L.HEOM_SOLVE_FP64, "fp32_ir": L.HEOM_SOLVE_FP32_IR, "shifted": L.HEOM_SOLVE_SHIFTED}


def solver_opts(**kw):
    """heom_solver_opts from keyword overrides of the library defaults
    (restart, max_iter, tol, precond, mode, inner_tol, max_refine, rhs_chunk,
    nn, fallback, use_x0, deflate)."""
    o = L.heom_solver_opts()
    lib().heom_default_opts(C.byref(o))
    for k, v in kw.items():
        if k == "precond":
            v = _PREC[v] if isinstance(v, str) else v
        elif k == "mode":
            v = _MODE[v] if isinstance(v, str) else v
        elif k == "nn":
            v = C.c_void_p(v.handle.value) if v is not None else None
        if not hasattr(o, k):
            raise TypeError(f"unknown solver option {k!r}")
        setattr(o, k, v)
    return o


def report_dict(r):
    return {f: getattr(r, f) for f, _ in L.heom_solver_report._fields_}


def _workspace(h, op, opts, n_rhs=1):
    import torch
    nbytes = C.c_size_t()
    L.check(lib().heom_workspace_size(h.handle, op, C.byref(opts) if opts is not None else None, n_rhs,
                                      C.byref(nbytes)))
    return torch.empty(max(int(nbytes.value), 1), dtype=torch.uint8, device="cuda")


def propagate(h, x, dt, n_steps, save_every=0, graph_steps=0, stream=None, ws=None):
    """RK4 in place on the device vector x; returns the trajectory of ADO 0
    ([n_steps // save_every][d][d]) when save_every > 0."""
    import torch
    prec = _precision_of(x)
    traj = None
    if save_every:
        traj = torch.empty((n_steps // save_every, h.d, h.d), dtype=x.dtype, device=x.device)
    if ws is None:
        ws = _workspace(h, L.HEOM_OP_PROPAGATE, None)
    L.check(lib().heom_propagate(h.handle, prec, _devptr(x), float(dt), int(n_steps), int(save_every),
                                 _devptr(traj) if traj is not None else None, int(graph_steps),
                                 C.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream)))
    return traj


def propagate_driven(h, x, dt, n_steps, drives, f, t0=0.0, save_every=0, stream=None, ws=None):
    """RK4 in place with H_s(t) = H + sum_k f(t)[k] drives[k]; f is a Python
    callable t -> sequence of len(drives) real coefficients.  Returns the
    trajectory of ADO 0 when save_every > 0."""
    import torch
    prec = _precision_of(x)
    V = [_c128(v) for v in drives]
    arr = np.ascontiguousarray(np.stack(V)).view(np.float64)
    traj = None
    if save_every:
        traj = torch.empty((n_steps // save_every, h.d, h.d), dtype=x.dtype, device=x.device)
    if ws is None:
        ws = _workspace(h, L.HEOM_OP_PROPAGATE, None)
    nd = len(V)

    def cb(t, out, _ctx):
        c = f(t)
        for i in range(nd):
            out[i] = float(c[i])

    fn = L.heom_drive_fn(cb)                      # kept alive for the duration of the call
    L.check(lib().heom_propagate_driven(h.handle, prec, _devptr(x), float(t0), float(dt), int(n_steps),
                                        int(save_every), _devptr(traj) if traj is not None else None, nd,
                                        arr.ctypes.data_as(L.dp), fn, None, C.c_void_p(ws.data_ptr()), ws.numel(),
                                        _stream_ptr(stream)))
    return traj


def steady_residual(h, x, r=None, stream=None):
    """r = e_0 - B x on the device (B the stationary-state operator)."""
    import torch
    if r is None:
        r = torch.empty_like(x)
    L.check(lib().heom_steady_residual(h.handle, _devptr(x), _devptr(r), _stream_ptr(stream)))
    return r


def axpby(x, alpha, y, beta, stream=None):
    """y = alpha x + beta y on the device (library kernel)."""
    L.check(lib().heom_vector_axpby(_precision_of(x), _devptr(x), float(alpha), _devptr(y), float(beta), x.numel(),
                                    _stream_ptr(stream)))
    return y


def current(h, x, lead, stream=None):
    """Electronic current (eq:last, e = hbar = 1) from the lead made of the
    fermionic bath records `lead` (indices into the hierarchy's bath list)
    into the system, read from the FP64 ADO vector x (complex)."""
    import torch
    if x.dtype != torch.complex128:
        raise TypeError("the current is read from an FP64 (complex128) ADO vector")
    if x.numel() != h.N * h.d * h.d:
        raise ValueError("x has the wrong size for this hierarchy")
    rec = np.ascontiguousarray(np.asarray(list(lead), dtype=np.int32))
    out = np.zeros(2)
    L.check(lib().heom_current(h.handle, _devptr(x), int(rec.size), rec.ctypes.data_as(L.i32p),
                               out.ctypes.data_as(L.dp), _stream_ptr(stream)))
    return complex(out[0], out[1])


def precondition(h, r, precond="block", shifts=None, n_rhs=1, border=False, stream=None):
    """z = P^{-1} r for a fixed preconditioner ('jacobi', 'scaled', 'block');
    r: [N][d][d] or [N][d][d][n_rhs] complex device tensor; shifts: optional
    tensor of n_rhs complex shifts (passed to the library as complex128)."""
    import torch
    z = torch.empty_like(r)
    R = int(n_rhs)
    if r.numel() != h.N * h.d * h.d * R:
        raise ValueError("r has the wrong size for this hierarchy")
    p = _PREC[precond] if isinstance(precond, str) else precond
    sh = None
    if shifts is not None:
        sh = shifts.to(device=r.device, dtype=torch.complex128).contiguous()
        if sh.numel() != R:
            raise ValueError("one shift per column")
    L.check(lib().heom_precondition(h.handle, _precision_of(r), int(p), _devptr(r), _devptr(z), int(R),
                                    _devptr(sh) if sh is not None else None, int(bool(border)), _stream_ptr(stream)))
    return z


def steady_state(h, x=None, stream=None, allow_not_converged=False, **opts):
    """Stationary ADOs (FP64 [N][d][d] device tensor) and the solver report.
    With allow_not_converged the iterate is returned when the solver stops
    at max_iter (report status 4)."""
    import torch
    o = solver_opts(**opts)
    if x is None:
        x = torch.zeros((h.N, h.d, h.d), dtype=torch.complex128, device="cuda")
    ws = _workspace(h, L.HEOM_OP_STEADY, o)
    rep = L.heom_solver_report()
    st = lib().heom_steady(h.handle, _devptr(x), C.byref(o), C.byref(rep), C.c_void_p(ws.data_ptr()), ws.numel(),
                           _stream_ptr(stream))
    if not (allow_not_converged and st == 4):
        L.check(st)
    return x, report_dict(rep)


def collect_pairs(h, net, snapshots=(10, 30, 60), x_star=None, restart=60, tol=1e-11, precond="none", stream=None):
    """Training pairs from plain GMRES runs (no preconditioner by default) on
    the stationary-state system: the converged x*, then iterates x_k after k
    iterations; for each snapshot the residual r = e_0 - B x_k and the error
    e = x* - x_k give one pair per ADO block.  Returns a list of (X, T, W)
    device tensors (W: row weights, see heom_nn_pairs)."""
    if x_star is None:
        x_star, _ = steady_state(h, tol=tol, restart=restart, max_iter=20000, precond=precond, stream=stream)
    out = []
    for k in snapshots:
        xk, _ = steady_state(h, restart=restart, max_iter=int(k), precond=precond, allow_not_converged=True,
                             stream=stream)
        r = steady_residual(h, xk, stream=stream)
        e = axpby(x_star, 1.0, xk, -1.0, stream=stream)   # e = x* - x_k (in place of x_k)
        out.append(net.pairs(h, r, e, border=1, stream=stream))
    return out


def spectrum(even, odd, x_ss, op, omegas, kind="dos", stream=None, allow_not_converged=False, **opts):
    """Density of states (kind 'dos', odd-parity `odd`) or power spectral
    density (kind 'psd') of operator `op` at the given frequencies.

    opts are solver options (solver_opts).  mode='shifted' with
    precond='none' serves every frequency from one Krylov space (multi-shift
    FOM; deflate=k > 0 adds thick restarts keeping k Schur vectors); the other
    modes solve per frequency, rhs_chunk frequencies per multi-RHS solve
    (0, the default, lets the library choose from the hierarchy size).  With
    allow_not_converged the values are returned when some frequency misses
    the tolerance (report status 4)."""
    o = solver_opts(**opts)
    om = np.ascontiguousarray(np.asarray(omegas, dtype=np.float64))
    out = np.zeros(len(om))
    k = 0 if kind == "dos" else 1
    hs = odd if k == 0 else even
    chunk = lib().heom_spectrum_chunk(hs.handle, C.byref(o))
    cols = max(1, min(chunk, len(om))) * (2 if k == 0 else 1)
    ws = _workspace(hs, L.HEOM_OP_SPECTRUM, o, cols)
    opm = _c128(op)
    rep = L.heom_solver_report()
    st = lib().heom_spectrum(even.handle, odd.handle if odd is not None else None, _devptr(x_ss), k, _dptr(opm),
                             _dptr(om), len(om), _dptr(out), C.byref(o), C.byref(rep),
                             C.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream))
    if not (allow_not_converged and st == 4):
        L.check(st)
    return out, report_dict(rep)


# ----------------------------------------------------------------- learned preconditioner
class Network:
    """Handle of heom_nn_create / heom_nn_load (see include/heom.h)."""

    def __init__(self, d=None, hidden=256, seed=0, path=None):
        self._lib = lib()
        h = C.c_void_p()
        if path is not None:
            L.check(self._lib.heom_nn_load(str(path).encode(), C.byref(h)))
        else:
            L.check(self._lib.heom_nn_create(int(d), int(hidden), int(seed), C.byref(h)))
        self._h = h
        k1, o_pad, n_params = C.c_int32(), C.c_int32(), C.c_int32()
        L.check(self._lib.heom_nn_info(h, C.byref(k1), C.byref(o_pad), C.byref(n_params)))
        self.k1, self.o_pad, self.n_params = k1.value, o_pad.value, n_params.value
        self.hidden = hidden

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            self._lib.heom_nn_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self):
        p = np.zeros(self.n_params, dtype=np.float32)
        L.check(self._lib.heom_nn_get_params(self._h, p.ctypes.data_as(C.POINTER(C.c_float))))
        return p

    def set_params(self, p):
        p = np.ascontiguousarray(np.asarray(p, dtype=np.float32))
        L.check(self._lib.heom_nn_set_params(self._h, p.ctypes.data_as(C.POINTER(C.c_float))))

    def save(self, path):
        L.check(self._lib.heom_nn_save(self._h, str(path).encode()))

    def pairs(self, h, r, e=None, border=1, stream=None):
        """(X bf16-as-int16 [N][k1], T fp32 [N][o_pad], W fp32 [N]) device
        tensors (T and W are None without e)."""
        import torch
        X = torch.empty((h.N, self.k1), dtype=torch.int16, device="cuda")
        T = torch.empty((h.N, self.o_pad), dtype=torch.float32, device="cuda") if e is not None else None
        W = torch.empty((h.N,), dtype=torch.float32, device="cuda") if e is not None else None
        L.check(self._lib.heom_nn_pairs(h.handle, self._h, _devptr(r), _devptr(e) if e is not None else None, border,
                                        _devptr(X), _devptr(T) if T is not None else None,
                                        _devptr(W) if W is not None else None, _stream_ptr(stream)))
        return X, T, W

    def forward(self, X, stream=None):
        import torch
        O = torch.empty((X.shape[0], self.o_pad), dtype=torch.float32, device="cuda")
        L.check(self._lib.heom_nn_forward(self._h, _devptr(X), X.shape[0], _devptr(O), _stream_ptr(stream)))
        return O

    def gradients(self, X, T, W=None, stream=None):
        g = np.zeros(self.n_params, dtype=np.float32)
        loss = C.c_float()
        L.check(self._lib.heom_nn_gradients(self._h, _devptr(X), _devptr(T), _devptr(W) if W is not None else None,
                                            X.shape[0],
                                            g.ctypes.data_as(C.POINTER(C.c_float)), C.byref(loss),
                                            _stream_ptr(stream)))
        return g, loss.value

    def train(self, X, T, W=None, epochs=10, batch=4096, lr=1e-3, seed=0, subset=0, stream=None):
        losses = np.zeros(max(epochs, 1), dtype=np.float32)
        L.check(self._lib.heom_nn_train(self._h, _devptr(X), _devptr(T), _devptr(W) if W is not None else None,
                                        X.shape[0], int(subset), epochs, batch,
                                        float(lr),
                                        int(seed), losses.ctypes.data_as(C.POINTER(C.c_float)), _stream_ptr(stream)))
        return losses[:epochs]


# ----------------------------------------------------------------- batched instances
class Batch:
    """Handle of heom_batch_create over already-built Hierarchy objects
    (kept alive by the batch).  Batch vectors are the instance vectors
    concatenated in order; ``offsets`` gives each instance's element range."""

    def __init__(self, hierarchies):
        self._lib = lib()
        self.members = list(hierarchies)
        arr = (C.c_void_p * len(self.members))(*[h.handle.value if isinstance(h.handle, C.c_void_p) else h.handle
                                                  for h in self.members])
        hb = C.c_void_p()
        L.check(self._lib.heom_batch_create(len(self.members), arr, C.byref(hb)))
        self._h = hb
        self.offsets = self.info()["offsets"]
        self.n = int(self.offsets[-1])

    def info(self):
        S = len(self.members)
        off = (C.c_int64 * (S + 1))()
        nt, grid, order = C.c_int64(), C.c_int32(), C.c_int32()
        L.check(self._lib.heom_batch_info(self._h, off, C.byref(nt), C.byref(grid), C.byref(order)))
        return {"offsets": np.array(off[:], dtype=np.int64), "n_tiles": nt.value, "grid": grid.value,
                "order": order.value}

    def close(self):
        if self._h:
            self._lib.heom_batch_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def split(self, v):
        """Views of the instance blocks [N_s][d_s][d_s] of a flat batch vector."""
        out = []
        for s, h in enumerate(self.members):
            a, b = int(self.offsets[s]), int(self.offsets[s + 1])
            out.append(v[a:b].view(h.N, h.d, h.d))
        return out

    def currents(self, x, lead, stream=None):
        """Electronic current (eq:last) from the lead `lead` (bath record
        indices, the same in every instance) of every instance of the FP64
        batch vector x."""
        return [current(h, v, lead, stream=stream) for h, v in zip(self.members, self.split(x))]

    def apply(self, x, y=None, border=0, stream=None):
        import torch
        if y is None:
            y = torch.empty_like(x)
        L.check(self._lib.heom_batch_apply(self._h, _precision_of(x), _devptr(x), _devptr(y), int(border),
                                           _stream_ptr(stream)))
        return y

    def tune(self, precision="fp32", reps=5, stream=None):
        import torch
        dt = torch.complex64 if precision == "fp32" else torch.complex128
        x = torch.randn(self.n, dtype=dt, device="cuda")
        y = torch.empty_like(x)
        md, mb = C.c_double(), C.c_double()
        L.check(self._lib.heom_batch_tune(self._h, _precision_of(x), _devptr(x), _devptr(y), int(reps),
                                          C.byref(md), C.byref(mb), _stream_ptr(stream)))
        return {"ms_default": md.value, "ms_best": mb.value, **self.info(), "shape": self.shape()}

    def shape(self):
        """The launch shape in use (heom_batch_shape)."""
        v = np.zeros(8, dtype=np.int32)
        L.check(self._lib.heom_batch_shape(self._h, v.ctypes.data_as(L.i32p)))
        keys = ("mult_small", "mult_wave", "var8", "var16", "grid", "order", "mfma16", "from_cache")
        return {k: int(x) for k, x in zip(keys, v)}

    def set_shape(self, mult_small=1, mult_wave=1, var8=1, var16=1, grid=0, order=0, mfma16=0):
        """Sets the launch shape (heom_batch_set_shape)."""
        v = np.array([mult_small, mult_wave, var8, var16, grid, order, mfma16], dtype=np.int32)
        L.check(self._lib.heom_batch_set_shape(self._h, v.ctypes.data_as(L.i32p)))

    def steady_state(self, x=None, use_graph=True, stream=None, allow_not_converged=False, **opts):
        """Stationary states of every instance: (FP64 batch vector, list of
        per-instance reports)."""
        import torch
        o = solver_opts(**opts)
        if x is None:
            x = torch.zeros(self.n, dtype=torch.complex128, device="cuda")
        nb = C.c_size_t()
        L.check(self._lib.heom_batch_workspace_size(self._h, C.byref(o), C.byref(nb)))
        ws = torch.empty(max(1, nb.value), dtype=torch.uint8, device="cuda")
        S = len(self.members)
        reps = (L.heom_solver_report * S)()
        st = self._lib.heom_batch_steady(self._h, _devptr(x), C.byref(o), reps, int(bool(use_graph)),
                                         C.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream))
        if not (allow_not_converged and st == 4):
            L.check(st)
        return x, [report_dict(r) for r in reps]
