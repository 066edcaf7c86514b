"""GPU parity of propagation, stationary state and spectra against the
oracle (RK4 on the assembled HEOMLS, sparse LU) and closed forms.

Bars: RK4 trajectories <= 1e-12 relative (FP64) / 1e-5 (FP32); linear
solves are run to a 1e-12 relative true residual and compared with the LU
solution to 1e-9 (the error is then set by the conditioning, stated in the
assertion messages); spectra of the U = 0 level match the closed form.
"""
import numpy as np
import pytest

from oracle import solvers as osv
from oracle.liouvillian import from_blocks, to_blocks
from paper_2306_07522_amd import workloads as wl
from tests.helpers import library_model, oracle_model, oracle_to_library_perm, rel_err

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def _api():
    from paper_2306_07522_amd import api
    return api


def _initial(om, lm, perm, rho0):
    xo = np.zeros((om.N, om.d, om.d), dtype=complex)
    xo[0] = rho0
    xl = np.zeros_like(xo)
    xl[perm] = xo
    return xo, xl


@pytest.mark.parametrize("graph", [0, 100])
def test_rk4_spin_boson(graph):
    torch, api = _torch(), _api()
    cfg = wl.spin_boson()
    om, lm = oracle_model(cfg), library_model(cfg)
    perm = oracle_to_library_perm(om, lm)
    xo, xl = _initial(om, lm, perm, cfg["rho0"])
    x = torch.from_numpy(xl).cuda()
    traj = api.propagate(lm, x, cfg["dt"], cfg["n_steps"], save_every=100, graph_steps=graph)
    xo_f, traj_o = osv.rk4(om.assemble(), from_blocks(xo), cfg["dt"], cfg["n_steps"], save_every=100, d=2)
    e_x = rel_err(x.cpu().numpy()[perm], to_blocks(xo_f, om.N, om.d))
    e_t = rel_err(traj.cpu().numpy(), np.array(traj_o))
    assert e_x <= 1e-12 and e_t <= 1e-12, (e_x, e_t)
    r = traj.cpu().numpy()
    assert np.abs(np.trace(r, axis1=1, axis2=2) - 1).max() < 1e-12
    assert np.abs(r - np.conj(np.transpose(r, (0, 2, 1)))).max() < 1e-12
    # FP32 trajectory against the FP64 oracle
    x32 = torch.from_numpy(xl.astype(np.complex64)).cuda()
    traj32 = api.propagate(lm, x32, cfg["dt"], cfg["n_steps"], save_every=100, graph_steps=graph)
    e32 = rel_err(traj32.cpu().numpy().astype(complex), np.array(traj_o))
    assert e32 <= 1e-5, e32


def test_rk4_graph_equals_eager():
    torch, api = _torch(), _api()
    cfg = wl.siam(n_max=2)
    lm = library_model(cfg)
    rng = np.random.default_rng(0)
    x0 = wl.random_vector(rng, lm.N, lm.d)
    xa = torch.from_numpy(x0).cuda()
    xb = torch.from_numpy(x0).cuda()
    ta = api.propagate(lm, xa, 0.002, 60, save_every=20, graph_steps=0)
    tb = api.propagate(lm, xb, 0.002, 60, save_every=20, graph_steps=20)
    assert torch.equal(xa, xb) and torch.equal(ta, tb)


@pytest.mark.parametrize("name", ["charge_cavity", "two_orbital_small", "siam_tier1", "siam_tier2", "cavity_d20",
                                  "dense_h_d16"])
def test_rk4_workloads(name):
    """Every stage's apply ends in the RK4 epilogue (wave kernel for d = 8,
    16, 20; the matrix-core self group for a dense d = 16 H; cell kernel for
    the d = 4 tier-2 model; the one-workgroup kernel for the tier-1 model).
    FP64 against the oracle's RK4 at 1e-12, FP32 at 1e-5."""
    torch, api = _torch(), _api()
    if name == "dense_h_d16":                                     # d = 16, dense H: matrix-core self group
        rng = np.random.default_rng(71)
        H = rng.standard_normal((16, 16)) + 1j * rng.standard_normal((16, 16))
        H = (H + H.conj().T) / np.linalg.norm(H + H.conj().T, 2)
        baths = wl.random_raw_baths(rng, 16, n_bos_baths=1, n_bos_exp=2, n_ferm_baths=1, n_ferm_exp=2,
                                    dense_ops=False)
        cfg = dict(name="dense_h_d16", H=H, baths=baths, m_max=2, n_max=2)
    elif name == "siam_tier2":
        cfg = wl.siam(n_max=2)                                    # d = 4: cell kernel
    elif name == "charge_cavity":
        cfg = wl.charge_cavity(n_photon=4, n_bexp=3, n_fexp=3)   # d = 8: wave kernel with fused stages
    elif name == "siam_tier1":
        cfg = wl.siam(n_max=1)                                    # 41 ADOs x 16: one-workgroup RK4 kernel
    elif name == "cavity_d20":
        cfg = wl.charge_cavity(n_photon=10, n_bexp=2, n_fexp=2, m_max=1, n_max=1)  # d = 20: masked wave kernel
    else:
        cfg = wl.two_orbital_anderson(n_max=2)                    # d = 16: wave kernel with fused stages
    om, lm = oracle_model(cfg), library_model(cfg)
    perm = oracle_to_library_perm(om, lm)
    rng = np.random.default_rng(5)
    xo = wl.random_vector(rng, om.N, om.d) * 0.1
    xl = np.empty_like(xo)
    xl[perm] = xo
    x = torch.from_numpy(xl).cuda()
    api.propagate(lm, x, 0.01, 20)
    ref, _ = osv.rk4(om.assemble(), from_blocks(xo), 0.01, 20)
    e = rel_err(x.cpu().numpy()[perm], to_blocks(ref, om.N, om.d))
    assert e <= 1e-12, e
    x32 = torch.from_numpy(xl.astype(np.complex64)).cuda()
    api.propagate(lm, x32, 0.01, 20)
    e32 = rel_err(x32.cpu().numpy()[perm].astype(complex), to_blocks(ref, om.N, om.d))
    assert e32 <= 1e-5, e32


@pytest.mark.parametrize("name", ["two_orbital_small", "siam_tier2"])
def test_rk4_zero_step(name):
    """dt = 0 (where the fused stages' shift 2/dt does not exist) takes the
    unfused step, which leaves the state exactly as it was."""
    torch, api = _torch(), _api()
    cfg = wl.two_orbital_anderson(n_max=2) if name == "two_orbital_small" else wl.siam(n_max=2)
    lm = library_model(cfg)
    x0 = wl.random_vector(np.random.default_rng(6), lm.N, lm.d)
    for dt in (torch.complex128, torch.complex64):
        x = torch.from_numpy(x0).to(dt).cuda()
        ref = x.clone()
        api.propagate(lm, x, 0.0, 3)
        assert torch.equal(x, ref)


def _steady_check(cfg, mode, precond, tol_err, lu=True):
    torch, api = _torch(), _api()
    om, lm = oracle_model(cfg), library_model(cfg)
    perm = oracle_to_library_perm(om, lm)
    x, rep = api.steady_state(lm, tol=1e-12, mode=mode, precond=precond, restart=40, max_iter=4000)
    xl = x.cpu().numpy()[perm]
    assert rep["status"] == 0 and rep["true_residual"] <= 1e-12, rep
    r0 = xl[0]
    assert abs(np.trace(r0) - 1) < 1e-10
    assert np.abs(r0 - r0.conj().T).max() < 1e-9
    M = om.assemble()
    res = np.linalg.norm(M @ from_blocks(xl)) / np.linalg.norm(from_blocks(xl))
    assert res < 1e-9, res
    if lu:
        xs = to_blocks(osv.steady_state(M, om.d), om.N, om.d)
        e = rel_err(xl, xs)
        assert e <= tol_err, (e, rep)
    return rep


@pytest.mark.parametrize("precond", ["jacobi", "none", "scaled"])
def test_steady_spin_boson(precond):
    _steady_check(wl.spin_boson(), "fp64", precond, 1e-10)


@pytest.mark.parametrize("precond", ["none", "scaled"])
def test_steady_siam_other_preconditioners(precond):
    _steady_check(wl.siam(n_max=2), "fp64", precond, 1e-9)


@pytest.mark.parametrize("mode", ["fp64", "fp32_ir"])
def test_steady_siam(mode):
    _steady_check(wl.siam(n_max=2), mode, "jacobi", 1e-9)


def test_steady_siam_full_tier():
    # 10,701 ADOs: residual against the oracle's assembled matrix
    _steady_check(wl.siam(), "fp64", "jacobi", None, lu=False)


def _dos_closed_form(w, eps, Gamma, W, mus):
    sigma = sum((Gamma * W / 2) / (w - mu + 1j * W) for mu in mus)
    return -(1.0 / (w - eps - sigma)).imag / np.pi


@pytest.mark.parametrize("mode", ["fp64", "fp32_ir", "shifted"])
def test_dos_resonant_level_closed_form(mode):
    torch, api = _torch(), _api()
    cfg = wl.resonant_level(eps=0.3, n_exp=3, n_max=2)
    he, ho = library_model(cfg, +1), library_model(cfg, -1)
    x, rep = api.steady_state(he, tol=1e-12)
    om = np.linspace(-8, 8, 37)
    extra = dict(precond="none", restart=60) if mode == "shifted" else {}
    A, rep = api.spectrum(he, ho, x, cfg["dops"][0], om, kind="dos", tol=1e-11, mode=mode, rhs_chunk=16, **extra)
    exact = _dos_closed_form(om, 0.3, 2.0, 10.0, (1.0, -1.0))
    assert np.abs(A - exact).max() < 1e-8, (np.abs(A - exact).max(), rep)


@pytest.mark.parametrize("mode", ["fp64", "shifted", "shifted_thick"])
def test_dos_siam_vs_oracle(mode):
    """shifted_thick: multi-shift FOM(12) with thick restarts keeping 4 Schur
    vectors, so that many restarts happen before 1e-12."""
    torch, api = _torch(), _api()
    cfg = wl.siam(n_max=2)
    he, ho = library_model(cfg, +1), library_model(cfg, -1)
    oe, oo = oracle_model(cfg, +1), oracle_model(cfg, -1)
    x, _ = api.steady_state(he, tol=1e-12)
    om = np.array([-7.0, -5.0, -1.0, 0.0, 0.5, 5.0])
    extra = dict(precond="none", restart=60) if mode == "shifted" else {}
    if mode == "shifted_thick":
        mode, extra = "shifted", dict(precond="none", restart=12, deflate=4, max_iter=5000)
    A, rep = api.spectrum(he, ho, x, cfg["dops"][0], om, kind="dos", tol=1e-12, rhs_chunk=4, mode=mode, **extra)
    assert rep["true_residual"] <= 1e-11, rep
    if extra.get("deflate"):
        assert rep["restarts"] >= 6, rep
    xs = osv.steady_state(oe.assemble(), oe.d)
    Ao = osv.dos(oo.assemble(), xs, cfg["dops"][0], om, oe.N, oe.d)
    assert np.abs(A - Ao).max() <= 1e-9 * np.abs(Ao).max(), (A, Ao)


@pytest.mark.parametrize("mode", ["fp64", "shifted", "shifted_thick", "block"])
def test_psd_cavity_vs_oracle(mode):
    torch, api = _torch(), _api()
    cfg = wl.charge_cavity(n_photon=4, n_bexp=3, n_fexp=2, m_max=2, n_max=1, lam=0.2, gamma=1.0, T=1.0, Gamma=0.5)
    he = library_model(cfg, +1)
    oe = oracle_model(cfg, +1)
    x, _ = api.steady_state(he, tol=1e-12)
    # w = 0 is excluded: M is singular in the even sector (the stationary
    # state is its null vector) and <a> != 0 for this model
    om = np.linspace(0.25, 2.0, 8)
    extra = dict(precond="none", restart=60) if mode == "shifted" else {}
    if mode == "block":
        mode, extra = "fp64", dict(precond="block")
    if mode == "shifted_thick":
        mode, extra = "shifted", dict(precond="none", restart=10, deflate=3, max_iter=5000)
    S, rep = api.spectrum(he, None, x, cfg["aop"], om, kind="psd", tol=1e-12, rhs_chunk=5, mode=mode, **extra)
    assert rep["true_residual"] <= 1e-11, rep
    xs = osv.steady_state(oe.assemble(), oe.d)
    So = osv.psd(oe.assemble(), xs, cfg["aop"], om, oe.N, oe.d)
    assert np.abs(S - So).max() <= 1e-9 * np.abs(So).max(), (S, So)


@pytest.mark.parametrize("mode", ["fp64", "block"])
def test_psd_cavity_configured_bath_vs_oracle(mode):
    """The cavity emission spectrum with the bath parameters of the full
    charge-cavity workload (Drude-Lorentz lambda 0.01, gamma 0.1, T 0.1 as a
    J pole plus 3 Matsubara terms; leads Gamma 0.01, tier 2 each way), cut
    to 2 photons and 2 lead exponents so that the oracle's sparse LU stays
    within seconds.  The frequencies straddle the cavity resonance."""
    torch, api = _torch(), _api()
    cfg = wl.charge_cavity(n_photon=2, n_fexp=2)
    he = library_model(cfg, +1)
    oe = oracle_model(cfg, +1)
    x, _ = api.steady_state(he, tol=1e-12)
    om = np.array([0.5, 0.9, 0.95, 1.0, 1.05, 1.5])
    # the unpreconditioned shifted solver stalls here (lead width 0.01)
    extra = dict(precond="block") if mode == "block" else {}
    S, rep = api.spectrum(he, None, x, cfg["aop"], om, kind="psd", tol=1e-12, rhs_chunk=6, mode="fp64", **extra)
    assert rep["true_residual"] <= 1e-11, rep
    xs = osv.steady_state(oe.assemble(), oe.d)
    So = osv.psd(oe.assemble(), xs, cfg["aop"], om, oe.N, oe.d)
    assert np.abs(S - So).max() <= 1e-9 * np.abs(So).max(), (S, So)


@pytest.mark.parametrize("restart,deflate", [(12, 4), (60, 0), (60, 8)])
def test_dos_invariant_krylov_space_vs_oracle(restart, deflate):
    """A 36-element odd hierarchy (resonant level, two exponents per lead,
    tier 1). FOM(12) keeping 4 Schur vectors exhausts the space after a few
    thick restarts. FOM(60) exhausts it within its first cycle. The Arnoldi
    breakdown then ends the solve with the exact projected solutions."""
    torch, api = _torch(), _api()
    cfg = wl.resonant_level(eps=0.3, n_exp=2, n_max=1)
    he, ho = library_model(cfg, +1), library_model(cfg, -1)
    oe, oo = oracle_model(cfg, +1), oracle_model(cfg, -1)
    assert ho.N * ho.d * ho.d == 36
    x, _ = api.steady_state(he, tol=1e-12)
    om = np.linspace(-6.0, 6.0, 25)
    A, rep = api.spectrum(he, ho, x, cfg["dops"][0], om, kind="dos", tol=1e-12, mode="shifted", precond="none",
                          restart=restart, deflate=deflate, max_iter=2000)
    assert rep["status"] == 0 and rep["true_residual"] <= 1e-11, rep
    xs = osv.steady_state(oe.assemble(), oe.d)
    Ao = osv.dos(oo.assemble(), xs, cfg["dops"][0], om, oe.N, oe.d)
    assert np.abs(A - Ao).max() <= 1e-9 * np.abs(Ao).max(), np.abs(A - Ao).max()


def test_dos_thick_restarts_report_an_iteration_cap():
    """With max_iter far too small the multi-shift solve reports status 4
    (not converged) and a residual above the tolerance. It raises, unless the
    caller accepts unconverged values."""
    torch, api = _torch(), _api()
    from paper_2306_07522_amd import _lib as L
    cfg = wl.siam(n_max=2)
    he, ho = library_model(cfg, +1), library_model(cfg, -1)
    x, _ = api.steady_state(he, tol=1e-12)
    om = np.linspace(-8.0, 8.0, 64)
    A, rep = api.spectrum(he, ho, x, cfg["dops"][0], om, kind="dos", tol=1e-12, mode="shifted", precond="none",
                          restart=12, deflate=4, max_iter=30, allow_not_converged=True)
    assert rep["status"] == 4 and rep["true_residual"] > 1e-12, rep
    assert rep["iterations"] <= 2 * 30, rep                 # two systems, each capped
    assert np.all(np.isfinite(A))
    with pytest.raises(L.HeomError):
        api.spectrum(he, ho, x, cfg["dops"][0], om, kind="dos", tol=1e-12, mode="shifted", precond="none",
                     restart=12, deflate=4, max_iter=30)


def test_dos_thick_restarts_match_plain_restarts_with_fewer_iterations():
    """Tier-3 SIAM (10,701 ADOs), 2,000 frequencies: the multi-shift solve
    with thick restarts (FOM(20), 6 Schur vectors kept) gives the plain
    FOM(40) density of states to the solver tolerance in fewer Arnoldi steps;
    on an evenly spaced sample, both match the per-frequency Jacobi-GMRES
    solve."""
    torch, api = _torch(), _api()
    cfg = wl.siam()
    he, ho = library_model(cfg, +1), library_model(cfg, -1)
    x, _ = api.steady_state(he, tol=1e-10, restart=60, max_iter=5000)
    om = cfg["omegas"]
    A0, r0 = api.spectrum(he, ho, x, cfg["dops"][0], om, kind="dos", tol=1e-8, mode="shifted", precond="none",
                          restart=40, max_iter=5000)
    A1, r1 = api.spectrum(he, ho, x, cfg["dops"][0], om, kind="dos", tol=1e-8, mode="shifted", precond="none",
                          restart=20, deflate=6, max_iter=5000)
    assert r0["status"] == 0 and r1["status"] == 0, (r0, r1)
    assert r1["true_residual"] <= 1e-8, r1
    scale = np.abs(A0).max()
    assert np.abs(A1 - A0).max() <= 1e-6 * scale, np.abs(A1 - A0).max()
    assert r1["iterations"] < r0["iterations"], (r0["iterations"], r1["iterations"])
    idx = np.linspace(0, len(om) - 1, 16).astype(int)
    As, rs = api.spectrum(he, ho, x, cfg["dops"][0], om[idx], kind="dos", tol=1e-10, rhs_chunk=16, precond="jacobi")
    assert np.abs(A1[idx] - As).max() <= 1e-6 * scale, np.abs(A1[idx] - As).max()


def test_steady_pruned_hierarchy_vs_oracle():
    """Stationary state of an importance-pruned hierarchy (eq:importance)
    against the oracle's direct solve of the pruned HEOMLS."""
    torch, api = _torch(), _api()
    from oracle import exponents as ox
    from oracle.liouvillian import OracleHEOM
    cfg = wl.siam(n_max=3, n_exp=3)
    th = 3e-3
    om = OracleHEOM(cfg["H"], ox.exponent_records(cfg["baths"]), 0, 3, importance_threshold=th)
    lm = api.Hierarchy(cfg["H"], cfg["baths"], 0, 3, parity_op=cfg["parity_op"], importance_threshold=th)
    perm = oracle_to_library_perm(om, lm)
    x, rep = api.steady_state(lm, tol=1e-12, restart=40, max_iter=4000)
    assert rep["status"] == 0, rep
    xs = to_blocks(osv.steady_state(om.assemble(), om.d), om.N, om.d)
    assert rel_err(x.cpu().numpy()[perm], xs) <= 1e-9


# ---------------------------------------------------------------- block preconditioner, deflated restarts
def _block_reference(x, H, decay, delta, shifts):
    """U ((U^H X U) / D) U^H per ADO and column, D = -(c_a - z) - i(E_i - E_j),
    |D| < delta -> -delta; x: [N][d][d][R]."""
    E, U = np.linalg.eigh(H)
    Xt = np.einsum("ki,akjr,jl->ailr", U.conj(), x, U)
    D = -(decay[:, None, None, None] - shifts[None, None, None, :]) - 1j * (E[None, :, None, None] - E[None, None, :, None])
    D = np.where(np.abs(D) < delta, -delta, D)
    return np.einsum("ik,aklr,jl->aijr", U, Xt / D, U.conj())


def _block_cfgs():
    return {
        "weak_cavity": wl.charge_cavity(n_photon=3, n_bexp=2, n_fexp=2),
        "two_orbital": wl.two_orbital_anderson(n_max=2),
        "siam": wl.siam(n_max=2, n_exp=2),
    }


@pytest.mark.parametrize("name", ["weak_cavity", "two_orbital", "siam"])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_block_preconditioner_matches_numpy(name, dtype):
    """heom_precondition(HEOM_PREC_BLOCK) against the eigenbasis formula in
    numpy, three columns with their own shifts (FP64 1e-12, FP32 1e-5)."""
    torch, api = _torch(), _api()
    cfg = _block_cfgs()[name]
    lm = library_model(cfg, parity_op=cfg.get("parity_op"))
    T = lm.tables()
    _, _, lev = lm.ados()
    tier1 = lev.sum(axis=1) == 1
    delta = T["decay"][tier1].real.min()
    R = 3
    rng = np.random.default_rng(3)
    x = rng.standard_normal((lm.N, lm.d, lm.d, R)) + 1j * rng.standard_normal((lm.N, lm.d, lm.d, R))
    shifts = np.array([0.0, 0.7j, -1.3 + 0.2j])
    if dtype == "c64":
        x = x.astype(np.complex64).astype(np.complex128)
    ref = _block_reference(x, cfg["H"], T["decay"], delta, shifts)
    xt = torch.from_numpy(x.astype(np.complex64) if dtype == "c64" else x).cuda()
    z = api.precondition(lm, xt, "block", shifts=torch.from_numpy(shifts).cuda(), n_rhs=R).cpu().numpy()
    tol = 1e-12 if dtype == "c128" else 1e-5
    assert rel_err(z.astype(np.complex128), ref) <= tol


def test_steady_block_preconditioner_weak_cavity():
    """A weakly damped cavity (Gamma = lambda = 0.01): restarted GMRES without
    a preconditioner stalls; with the block preconditioner it converges in
    a few cycles, to the oracle's LU solution."""
    torch, api = _torch(), _api()
    cfg = wl.charge_cavity(n_photon=3, n_bexp=2, n_fexp=2)
    om, lm = oracle_model(cfg), library_model(cfg, parity_op=cfg["parity_op"])
    perm = oracle_to_library_perm(om, lm)
    xs = to_blocks(osv.steady_state(om.assemble(), om.d), om.N, om.d)
    x, rep = api.steady_state(lm, tol=1e-12, precond="block", restart=30, max_iter=600)
    assert rep["status"] == 0 and rep["iterations"] <= 300, rep
    assert rel_err(x.cpu().numpy()[perm], xs) <= 1e-9
    _, rep0 = api.steady_state(lm, tol=1e-8, precond="none", restart=30, max_iter=600, allow_not_converged=True)
    assert rep0["status"] == 4, rep0


@pytest.mark.parametrize("mode", ["fp64", "fp32_ir"])
@pytest.mark.parametrize("precond", ["none", "block"])
def test_steady_deflated_restarting_vs_oracle(mode, precond):
    """GMRES-DR (deflated restarts) reaches the oracle's LU solution.  Without
    a preconditioner, on a short restart length, it needs no more iterations
    than plain restarts (with the block preconditioner the spectrum is
    already clustered and keeping k of m vectors need not pay)."""
    torch, api = _torch(), _api()
    cfg = wl.siam(n_max=2, n_exp=2)
    om, lm = oracle_model(cfg), library_model(cfg, parity_op=cfg["parity_op"])
    perm = oracle_to_library_perm(om, lm)
    xs = to_blocks(osv.steady_state(om.assemble(), om.d), om.N, om.d)
    kw = dict(tol=1e-11, precond=precond, restart=10, max_iter=6000, mode=mode)
    x, rep = api.steady_state(lm, deflate=4, **kw)
    assert rep["status"] == 0, rep
    assert rel_err(x.cpu().numpy()[perm], xs) <= 1e-8
    _, rep0 = api.steady_state(lm, **kw)
    assert rep0["status"] == 0, rep0
    if mode == "fp64" and precond == "none":
        assert rep["iterations"] <= rep0["iterations"], (rep, rep0)


def test_steady_deflated_weak_cavity_vs_oracle():
    """GMRES-DR with the block preconditioner on the weak cavity."""
    torch, api = _torch(), _api()
    cfg = wl.charge_cavity(n_photon=3, n_bexp=2, n_fexp=2)
    om, lm = oracle_model(cfg), library_model(cfg, parity_op=cfg["parity_op"])
    perm = oracle_to_library_perm(om, lm)
    xs = to_blocks(osv.steady_state(om.assemble(), om.d), om.N, om.d)
    x, rep = api.steady_state(lm, tol=1e-12, precond="block", restart=20, deflate=6, max_iter=600)
    assert rep["status"] == 0, rep
    assert rel_err(x.cpu().numpy()[perm], xs) <= 1e-9


# ---------------------------------------------------------------- full sizes, sampled oracle rows
def _sampled_steady_residual(om, xo, per_tier, seed):
    """b - B x on a seeded sample of block rows of the oracle's bordered
    operator (every tier represented, ADO 0 included), B x from the oracle's
    assembled rows applied to the library's solution (oracle order)."""
    rng = np.random.default_rng(seed)
    lev = np.array([len(j) + len(q) for j, q in om.hier.ados])
    rows = [0]
    for t in range(1, lev.max() + 1):
        cand = np.nonzero(lev == t)[0]
        rows += rng.choice(cand, min(per_tier, len(cand)), replace=False).tolist()
    d = om.d
    y = (om.assemble(rows=rows) @ from_blocks(xo)).reshape(len(rows), d, d).transpose(0, 2, 1)
    y[0, 0, 0] = np.trace(xo[0])                      # the trace row of the bordered system
    b = np.zeros_like(y)
    b[0, 0, 0] = 1.0
    return np.linalg.norm((b - y).ravel())


def test_full_size_two_orbital_steady_state_on_sampled_oracle_rows():
    """Two-orbital tier 4 (213,053 ADOs) with GMRES-DR(20, 6): the solution
    satisfies the oracle's bordered equations on sampled rows."""
    torch, api = _torch(), _api()
    cfg = wl.two_orbital_anderson()
    om, lm = oracle_model(cfg), library_model(cfg, parity_op=cfg["parity_op"])
    perm = oracle_to_library_perm(om, lm)
    x, rep = api.steady_state(lm, tol=1e-9, precond="none", restart=20, deflate=6, max_iter=3000)
    assert rep["status"] == 0 and rep["true_residual"] <= 1e-9, rep
    xo = x.cpu().numpy()[perm]
    assert _sampled_steady_residual(om, xo, 80, 7) <= 2e-9
    rho = xo[0]
    assert abs(np.trace(rho) - 1.0) <= 1e-12 and np.abs(rho - rho.conj().T).max() <= 1e-9


def test_full_size_cavity_steady_state_on_sampled_oracle_rows():
    """Charge cavity (3,165 ADOs of 20 x 20) with the block preconditioner."""
    torch, api = _torch(), _api()
    cfg = wl.charge_cavity()
    om, lm = oracle_model(cfg), library_model(cfg, parity_op=cfg["parity_op"])
    perm = oracle_to_library_perm(om, lm)
    x, rep = api.steady_state(lm, tol=1e-10, precond="block", restart=60, max_iter=3000)
    assert rep["status"] == 0, rep
    xo = x.cpu().numpy()[perm]
    assert _sampled_steady_residual(om, xo, 60, 11) <= 2e-10
