"""The learned Newton guess on the GPU: the matrix-core forward and the training gradient against
the FP64 reference (oracle/mlp.py) on the same BF16-rounded weights, Adam against its formula,
and the guarantee that the guess never changes an inversion's result (Newton refines to the same
tolerance and the analytic guess rescues every failure)."""
import ctypes

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from oracle import mlp as M
from tests.parity import prim_errors

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def S():
    from paper_2012_11130_amd import srhd
    return srhd


def _net(S, theta, norm, features=0, gate=0.0):
    """Device parameters for a flat FP64 parameter vector (BF16 weights as the kernels read)."""
    p = M.unpack(theta)
    w = np.concatenate([p["W1"].ravel(), p["W2"].ravel(), p["W3"].ravel()]).astype(np.float32)
    wb = torch.from_numpy(w).to(torch.bfloat16).view(torch.int16).to(DEV)
    b = torch.from_numpy(np.concatenate([p["b1"], p["b2"], p["b3"]]).astype(np.float32)).to(DEV)
    return S.Mlp(wb.contiguous(), b, torch.tensor(norm, dtype=torch.float32, device=DEV), features, gate)


def _rand_theta(seed):
    rng = np.random.default_rng(seed)
    return M.init(seed) + 0.05 * rng.standard_normal(M.N_PARAM)


@pytest.mark.parametrize("n", [64, 1000, 100_003])
def test_forward_matches_reference(S, n):
    rng = np.random.default_rng(n)
    theta = _rand_theta(1)
    norm = np.array([0.1, -0.2, 0.3, 1.5, 2.0, 0.7, -3.0, 2.5])
    feat = rng.standard_normal((3, n)) * 3
    net = _net(S, theta, norm)
    y = S.srhd_mlp_forward(net, torch.from_numpy(feat.astype(np.float32)).to(DEV)).cpu().numpy()
    f32 = feat.astype(np.float32).astype(np.float64)
    x = (f32 - norm[:3, None]) / norm[3:6, None]
    z, _ = M.forward(M.pack(M.unpack(theta)), x, bf16_round=True)
    ref = norm[6] + norm[7] * z
    err = np.abs(y - ref)
    assert np.max(err) <= 2e-3 * (1 + np.max(np.abs(ref))), np.max(err)
    assert np.mean(err) <= 1e-4 * (1 + np.mean(np.abs(ref)))


def test_gradient_matches_reference(S):
    rng = np.random.default_rng(5)
    theta = _rand_theta(2)
    norm = np.array([0.0, 0.0, 0.0, 1.0, 1.0, 1.0, 0.5, 2.0])
    n = 4096
    feat = rng.standard_normal((3, n))
    target = rng.standard_normal(n) * 2 + 0.5
    net = _net(S, theta, norm)
    g, loss = S.srhd_mlp_grad(net, torch.from_numpy(feat.astype(np.float32)).to(DEV),
                              torch.from_numpy(target.astype(np.float32)).to(DEV))
    g = g.cpu().numpy().astype(np.float64)
    x = feat.astype(np.float32).astype(np.float64)
    t = (target.astype(np.float32).astype(np.float64) - norm[6]) / norm[7]
    # the reference on the same BF16-rounded weights
    p = M.unpack(theta)
    for k in ("W1", "W2", "W3"):
        p[k] = M.bf16(p[k])
    lr, gr = M.loss_and_grad(M.pack(p), x, t, bf16_round=True)
    assert abs(loss.item() / lr - 1) < 1e-4
    assert np.linalg.norm(g - gr) <= 1e-2 * np.linalg.norm(gr)
    for blk, (a, b) in {"W1": (0, 192), "W2": (256, 4352), "W3": (4416, 4480)}.items():
        assert np.linalg.norm(g[a:b] - gr[a:b]) <= 2e-2 * np.linalg.norm(gr[a:b]), blk
    # bit-reproducible
    g2, _ = S.srhd_mlp_grad(net, torch.from_numpy(feat.astype(np.float32)).to(DEV),
                            torch.from_numpy(target.astype(np.float32)).to(DEV))
    assert np.array_equal(g2.cpu().numpy(), g.astype(np.float32))


def test_adam_matches_formula(S):
    rng = np.random.default_rng(6)
    theta = rng.standard_normal(M.N_PARAM).astype(np.float32)
    m1 = (rng.standard_normal(M.N_PARAM) * 0.1).astype(np.float32)
    m2 = np.abs(rng.standard_normal(M.N_PARAM) * 0.01).astype(np.float32)
    g = rng.standard_normal(M.N_PARAM).astype(np.float32)
    net = _net(S, theta.astype(np.float64), np.array([0, 0, 0, 1, 1, 1, 0, 1.0]))
    t_, a_, b_ = (torch.from_numpy(v.copy()).to(DEV) for v in (theta, m1, m2))
    S.srhd_mlp_adam(t_, a_, b_, torch.from_numpy(g).to(DEV), 3, 1e-2, net)
    ref, rm, rv = M.adam(theta.astype(np.float64), g.astype(np.float64), m1.astype(np.float64),
                         m2.astype(np.float64), 3, 1e-2)
    assert np.allclose(t_.cpu().numpy(), ref, rtol=1e-5, atol=1e-6)
    assert np.allclose(a_.cpu().numpy(), rm, rtol=1e-5, atol=1e-7)
    # the BF16 copy the inference reads was refreshed
    wb = net.w.cpu().view(torch.bfloat16).float().numpy()
    assert np.allclose(wb[:192], M.bf16(ref[:192]), rtol=0, atol=0)


@pytest.mark.parametrize("kind", [0, 1])
def test_features_match_reference(S, kind):
    prim = W.conversion_batch(100_000, seed=44)
    cons = O.prim2cons(prim)
    cons[:, :50] = cons[:, 50:100] * np.array([[1.0], [1.0], [1.0], [1.0], [-1.0]])   # Et < 0
    ref = M.features(cons, kind)
    got, _ = S.srhd_mlp_features(torch.from_numpy(cons).to(DEV), features=kind)
    got = got.cpu().numpy().astype(np.float64)
    fin = np.isfinite(ref)
    assert np.array_equal(fin, np.isfinite(got))
    assert np.all(np.abs(got[fin] - ref[fin]) <= 2e-6 * (1 + np.abs(ref[fin])))


def test_learned_guess_never_changes_the_inversion(S):
    # a (random, untrained) network as the first guess: Newton + analytic fallback must return
    # the same primitives as the analytic guess alone, within the parity tolerance
    prim = W.conversion_batch(50_000, seed=41)
    cons = O.prim2cons(prim)
    ref, st_ref, _ = O.cons2prim(cons)
    f = M.features(cons)
    good = np.isfinite(f).all(axis=0)
    norm = np.concatenate([f[:, good].mean(axis=1), f[:, good].std(axis=1), [-5.0, 8.0]])
    net = _net(S, _rand_theta(3), norm)
    c = torch.from_numpy(cons).to(DEV)
    w, st, it = S.srhd_cons2prim(c, status=True, iters=True, guess=net.guess())
    w, st = w.cpu().numpy(), st.cpu().numpy()
    bad = st_ref == O.ST_UNPHYSICAL
    assert np.array_equal(st == S.ST_UNPHYSICAL, bad)
    assert set(np.unique(st[~bad])) <= {S.ST_OK, S.ST_FALLBACK}
    assert max(prim_errors(w, ref, ~bad).values()) <= 1e-12


def test_poisoned_network_falls_back_everywhere(S):
    prim = W.conversion_batch(10_000, seed=42)
    cons = O.prim2cons(prim)
    ref, st_ref, _ = O.cons2prim(cons)
    theta = _rand_theta(4)
    theta[300] = np.nan
    net = _net(S, theta, np.array([0, 0, 0, 1, 1, 1, 0, 1.0]))
    w, st, _ = S.srhd_cons2prim(torch.from_numpy(cons).to(DEV), status=True, guess=net.guess())
    st = st.cpu().numpy()
    ok = st_ref == 0
    assert np.all(st[ok] == S.ST_FALLBACK)
    assert max(prim_errors(w.cpu().numpy(), ref, ok).values()) <= 1e-12


@pytest.mark.parametrize("kind,gate", [(0, 0.0), (1, 0.1)])
def test_gated_guess_never_changes_the_inversion(S, kind, gate):
    # a random network consulted only above the gate: results as with the analytic guess, and
    # states at or below the gate never report a fallback
    prim = W.conversion_batch(50_000, seed=45)
    cons = O.prim2cons(prim)
    ref, st_ref, _ = O.cons2prim(cons)
    f = M.features(cons, kind)
    good = np.isfinite(f).all(axis=0)
    norm = np.concatenate([f[:, good].mean(axis=1), f[:, good].std(axis=1), [-5.0, 8.0]])
    net = _net(S, _rand_theta(6), norm, kind, gate)
    w, st, _ = S.srhd_cons2prim(torch.from_numpy(cons).to(DEV), status=True, guess=net.guess())
    w, st = w.cpu().numpy(), st.cpu().numpy()
    bad = st_ref == O.ST_UNPHYSICAL
    assert np.array_equal(st == S.ST_UNPHYSICAL, bad)
    assert max(prim_errors(w, ref, ~bad).values()) <= 1e-12
    L = O.L_batch(cons)
    if gate > 0:
        assert not np.any(st[(L <= gate) & ~bad] == S.ST_FALLBACK)


def test_step_with_learned_guess_matches_oracle(S):
    # the 64^3 blast, one step of the gather path with the network guessing every inversion
    from tests.parity import oracle_cons, step_errors
    g = W.blast(64, seed=3, order="morton")
    cons = oracle_cons(g)
    f = M.features(O.prim2cons(W.conversion_batch(20_000, seed=43)))
    norm = np.concatenate([f.mean(axis=1), f.std(axis=1), [-5.0, 8.0]])
    c = torch.from_numpy(cons).to(DEV)
    nb = torch.from_numpy(g.neighbor).to(DEV)
    dt_o, _, _ = O.cfl_dt(cons, None, g.dh_lev, 0.5)
    ref, _ = O.fluid_step(O.fill_ghosts(cons, g.neighbor, 3), dt_o, g.dh_lev)
    for prec, kind, gate in ((0, 0, 0.0), (1, 0, 0.0), (0, 1, 0.1), (1, 1, 0.1)):
        net = _net(S, _rand_theta(5), norm, kind, gate)
        prims, smax = S.srhd_grid_prims(c, prec=prec, guess=net.guess())
        st = S.new_stats(DEV)
        out, _, _ = S.srhd_fluid_step_grid(c, prims, nb, g.dh_lev, dt_lev=torch.from_numpy(dt_o).to(DEV),
                                           prec=prec, stats=st, guess=net.guess())
        e = step_errors(out.cpu().numpy(), ref)
        if prec == 0:
            assert max(e.values()) <= 1e-10, (prec, e)
        else:
            # the FP32 bulk's bound per patch (Eq. 20; tests/test_gpu_guard.py)
            from tests.parity import kappa_tile_padded, patch_errors, step_bound
            bound = step_bound(kappa_tile_padded(O.fill_ghosts(cons, g.neighbor, 3)))
            assert np.all(patch_errors(out.cpu().numpy(), ref) <= bound), (prec, e)
        sd = S.stats_dict(st)
        assert sd["n_noconv"] == 0 and sd["n_unphysical"] == 0
