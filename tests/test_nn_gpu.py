"""GPU parity of the learned preconditioner's kernels against the oracle
network, and its use inside FGMRES.

Bars: forward and gradients within 1e-2 of the largest element per layer and
1e-3 relative on norms (BF16 operands, FP32 accumulation, compared with the
oracle's BF16 emulation); features within one BF16 rounding; training on the
method's own (residual, error) pairs halves the held-out loss; FGMRES with the
network reaches the true-residual tolerance."""
import numpy as np
import pytest

from oracle import nn as onn
from oracle.liouvillian import from_blocks, to_blocks
from paper_2306_07522_amd import workloads as wl
from tests.helpers import library_model, oracle_model, oracle_to_library_perm

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def _api():
    from paper_2306_07522_amd import api
    return api


def _bits(x32):
    """float32 BF16-valued array -> int16 bit patterns (device tensor)."""
    torch = _torch()
    u = (np.ascontiguousarray(x32, dtype=np.float32).view(np.uint32) >> 16).astype(np.uint16).view(np.int16)
    return torch.from_numpy(u.copy()).cuda()


def _from_bits(t):
    u = t.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32)


def _layers(net):
    return onn.unpack(net.get_params().astype(np.float64), net.k1, net.hidden, net.o_pad)


def _close(a, b, name):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    scale = max(np.abs(b).max(), 1e-30)
    assert np.abs(a - b).max() <= 1e-2 * scale, (name, np.abs(a - b).max(), scale)
    assert abs(np.linalg.norm(a) - np.linalg.norm(b)) <= 1e-3 * np.linalg.norm(b) + 1e-30, name


@pytest.mark.parametrize("d,rows", [(4, 300), (16, 130)])
def test_forward_and_gradients_match_oracle(d, rows):
    torch, api = _torch(), _api()
    net = api.Network(d=d, hidden=64 if d == 4 else 256, seed=11)
    rng = np.random.default_rng(d)
    # make the last layer larger than its init so every path carries signal
    p = net.get_params()
    net.set_params(p + np.float32(0.05) * rng.standard_normal(p.size).astype(np.float32))
    X = onn.bf16(rng.standard_normal((rows, net.k1)).astype(np.float32))
    X[:, 2 * d * d + 6:] = 0
    T = rng.standard_normal((rows, net.o_pad)).astype(np.float32)
    W = rng.uniform(0.05, 3.0, rows).astype(np.float32)
    layers = _layers(net)
    O_ref, _ = onn.forward_bf16(layers, X)
    O = net.forward(_bits(X)).cpu().numpy()
    _close(O, O_ref, "forward")
    g, loss = net.gradients(_bits(X), torch.from_numpy(T).cuda(), torch.from_numpy(W).cuda())
    g_ref, loss_ref = onn.grads_bf16(layers, X, T, W)
    assert abs(loss - loss_ref) <= 1e-4 * abs(loss_ref)
    off = 0
    for l, (gW, gb) in enumerate(g_ref):
        nW = gW.size
        _close(g[off: off + nW].reshape(gW.shape), gW, f"dW{l + 1}")
        off += nW
        _close(g[off: off + gb.size], gb, f"db{l + 1}")
        off += gb.size


def test_features_and_targets_match_oracle():
    torch, api = _torch(), _api()
    cfg = wl.siam(n_max=2)
    om, lm = oracle_model(cfg), library_model(cfg)
    perm = oracle_to_library_perm(om, lm)
    net = api.Network(d=4, hidden=64, seed=1)
    rng = np.random.default_rng(3)
    r_o = wl.random_vector(rng, om.N, om.d)
    r_o[5] = 0  # a converged block
    e_o = wl.random_vector(rng, om.N, om.d)
    r_l, e_l = np.empty_like(r_o), np.empty_like(e_o)
    r_l[perm], e_l[perm] = r_o, e_o
    X, T, W = net.pairs(lm, torch.from_numpy(r_l).cuda(), torch.from_numpy(e_l).cuda())
    Xg = _from_bits(X)[perm]
    Tg = T.cpu().numpy()[perm]
    Wg = W.cpu().numpy()[perm]
    lev_n = np.array([len(q) for _, q in om.hier.ados])
    lev_m = np.array([len(j) for j, _ in om.hier.ados])
    decay = np.array([sum(om.ferm[x]["gamma"] for x in q) for _, q in om.hier.ados])
    Xo, nu = onn.features(r_o, lev_n, lev_m, decay, 2, 0, net.k1)
    assert np.abs(Xg - Xo).max() <= 2.0 ** -7 * max(1.0, np.abs(Xo).max())
    To, Wo = onn.targets(r_o, e_o)
    assert np.abs(Tg[:, : To.shape[1]] - To).max() <= 1e-5 * np.abs(To).max()
    assert np.all(Tg[:, To.shape[1]:] == 0)
    assert np.abs(Wg - Wo).max() <= 1e-5 * Wo.max()
    assert Wg[5] == 0 and np.all(Xg[5, : 2 * om.d * om.d] == 0)


def test_training_fits_a_learnable_map():
    """Adam over the hand-written forward/backward kernels fits a fixed
    linear map of the features (loss falls by 10x)."""
    torch, api = _torch(), _api()
    net = api.Network(d=4, hidden=64, seed=4)
    rng = np.random.default_rng(8)
    rows = 16384
    X = onn.bf16(rng.standard_normal((rows, net.k1)).astype(np.float32))
    X[:, 2 * 16 + 6:] = 0
    Mfix = rng.standard_normal((net.k1, net.o_pad)).astype(np.float32) / np.sqrt(36.0)
    T = (X @ Mfix).astype(np.float32)
    losses = net.train(_bits(X), torch.from_numpy(T).cuda(), epochs=40, batch=1024, lr=3e-3, seed=2)
    assert np.all(np.isfinite(losses))
    assert losses[-1] < 0.1 * losses[0], losses


def test_zero_network_is_the_identity():
    """z = r + nu * 0: FGMRES with a zero network is GMRES without a
    preconditioner, iteration for iteration."""
    torch, api = _torch(), _api()
    cfg = wl.siam()
    h = library_model(cfg, parity_op=cfg["parity_op"])
    net = api.Network(d=4, hidden=64, seed=0)
    net.set_params(np.zeros(net.n_params, dtype=np.float32))
    x_n, rep_n = api.steady_state(h, tol=1e-10, precond="nn", nn=net, fallback=0, restart=30, max_iter=3000)
    x_j, rep_j = api.steady_state(h, tol=1e-10, precond="none", restart=30, max_iter=3000)
    assert rep_n["iterations"] == rep_j["iterations"] and rep_n["fell_back"] == 0
    assert (x_n - x_j).abs().max().item() <= 1e-10 * x_j.abs().max().item()


def _siam_pairs(api, net, seeds, snapshots=(10, 30, 60)):
    """(X, T, W) from plain GMRES on seeded perturbations of the Anderson
    impurity model at tier 2 (eps, U, Gamma, mu each times e^{0.1 Z})."""
    import torch
    Xs, Ts, Ws = [], [], []
    for s in seeds:
        z = np.exp(0.1 * np.random.default_rng(s).standard_normal(4))
        pc = wl.siam(eps=-5.0 * z[0], U=10.0 * z[1], Gamma=2.0 * z[2], mus=(z[3], -z[3]), n_max=2)
        hp = library_model(pc, parity_op=pc["parity_op"])
        for X, T, W in api.collect_pairs(hp, net, snapshots=snapshots, restart=20):
            Xs.append(X)
            Ts.append(T)
            Ws.append(W)
        hp.close()
    return torch.cat(Xs), torch.cat(Ts), torch.cat(Ws)


def test_training_on_solver_pairs_halves_held_out_loss():
    """The network trained on (residual, error) pairs that plain GMRES
    generates on 16 seeded perturbations of the Anderson impurity model:
    the weighted loss on pairs from 4 other seeds (never trained on) falls
    by at least 2x from the untrained network's."""
    torch, api = _torch(), _api()
    net = api.Network(d=4, hidden=256, seed=3)
    Xtr, Ttr, Wtr = _siam_pairs(api, net, range(1000, 1016))
    Xte, Tte, Wte = _siam_pairs(api, net, range(2000, 2004))
    _, before = net.gradients(Xte, Tte, Wte)
    losses = net.train(Xtr, Ttr, Wtr, epochs=120, batch=1024, lr=1e-3, seed=7)
    _, after = net.gradients(Xte, Tte, Wte)
    print(f"\ntrain rows {Xtr.shape[0]}, held-out rows {Xte.shape[0]}: held-out loss {before:.4g} -> {after:.4g}; "
          f"training loss {losses[0]:.4g} -> {losses[-1]:.4g}")
    assert np.all(np.isfinite(losses))
    assert after <= 0.5 * before, (before, after)


def test_trained_network_in_fgmres():
    """Pairs from plain GMRES on perturbed models, GPU training, then the
    stationary state with the network: the answer is the unpreconditioned
    one to the true-residual tolerance, whether the network converges itself
    or hands over to Jacobi on stagnation.  Its gain is measured, not
    asserted."""
    torch, api = _torch(), _api()
    cfg = wl.siam(n_max=2)
    net = api.Network(d=4, hidden=128, seed=0)
    X, T, W = _siam_pairs(api, net, range(1000, 1004), snapshots=(10, 40))
    losses = net.train(X, T, W, epochs=8, batch=4096, lr=1e-3, seed=5)
    assert np.all(np.isfinite(losses))
    h = library_model(cfg, parity_op=cfg["parity_op"])
    x_nn, rep_nn = api.steady_state(h, tol=1e-10, precond="nn", nn=net, restart=30)
    x_0, rep_0 = api.steady_state(h, tol=1e-10, precond="none", restart=30, max_iter=5000)
    assert rep_nn["status"] == 0 and rep_nn["true_residual"] <= 1e-10, rep_nn
    assert (x_nn - x_0).abs().max().item() <= 1e-8 * x_0.abs().max().item()
    print(f"\nloss {losses[0]:.3g} -> {losses[-1]:.3g}; iterations nn {rep_nn['iterations']} "
          f"(fell back: {rep_nn['fell_back']}, {rep_nn['seconds']:.3f} s) / none {rep_0['iterations']} "
          f"({rep_0['seconds']:.3f} s)")


def test_nan_network_falls_back_to_jacobi():
    torch, api = _torch(), _api()
    cfg = wl.siam(n_max=2)
    h = library_model(cfg, parity_op=cfg["parity_op"])
    net = api.Network(d=4, hidden=64, seed=2)
    p = net.get_params()
    p[:] = np.nan
    net.set_params(p)
    x, rep = api.steady_state(h, tol=1e-10, precond="nn", nn=net, fallback=1)
    assert rep["fell_back"] == 1 and rep["status"] == 0 and rep["true_residual"] <= 1e-10, rep
    from paper_2306_07522_amd._lib import HeomError
    with pytest.raises(HeomError):
        api.steady_state(h, tol=1e-10, precond="nn", nn=net, fallback=0)


def test_save_load_roundtrip(tmp_path):
    api = _api()
    net = api.Network(d=4, hidden=64, seed=9)
    path = tmp_path / "net.bin"
    net.save(path)
    net2 = api.Network(path=path)
    assert np.array_equal(net.get_params(), net2.get_params())
