"""Pins of the FP64 surrogate reference (oracle/mlp.py) against things other
than itself: torch's autograd and its Adam optimiser (float64, CPU), central
finite differences, the C oracle's voxelization, and closed-form occupancy
cases."""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import mlp


def _rand_member(layers, seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, scale, mlp.n_params(layers))


def test_parameter_count():
    # 80*256+256 + 2*(256*256+256) + 256*17+17
    assert mlp.n_params() == 156689


def _torch_net(flat, layers):
    ps = [torch.tensor(W.copy(), requires_grad=True) for pair in mlp.unpack(flat, layers) for W in pair]

    def run(X):
        a = X
        for i in range(0, len(ps), 2):
            a = a @ ps[i].T + ps[i + 1]
            if i + 2 < len(ps):
                a = torch.nn.functional.silu(a)
        return a
    return ps, run


@pytest.mark.parametrize("layers", [(5, 7, 6, 3), mlp.LAYERS])
def test_forward_backward_match_torch_autograd(layers):
    w = _rand_member(layers, 1, 0.2)
    rng = np.random.default_rng(2)
    X = rng.normal(size=(9, layers[0]))
    T = rng.normal(size=(9, layers[-1]))
    Y, cache = mlp.forward(w, X, layers)
    g = mlp.backward(w, cache, Y, T, layers)
    ps, run = _torch_net(w, layers)
    Yt = run(torch.tensor(X))
    loss = ((Yt - torch.tensor(T)) ** 2).mean()
    loss.backward()
    gt = np.concatenate([p.grad.numpy().ravel() for p in ps])
    assert np.allclose(Y, Yt.detach().numpy(), rtol=1e-12, atol=1e-13)
    assert abs(mlp.mse(Y, T) - loss.item()) <= 1e-12 * loss.item()
    assert np.linalg.norm(g - gt) <= 1e-11 * np.linalg.norm(gt)


def test_backward_matches_central_differences():
    layers = (4, 6, 5, 2)
    w = _rand_member(layers, 3, 0.5)
    rng = np.random.default_rng(4)
    X = rng.normal(size=(7, 4))
    T = rng.normal(size=(7, 2))
    Y, cache = mlp.forward(w, X, layers)
    g = mlp.backward(w, cache, Y, T, layers)
    h = 1e-6
    fd = np.empty_like(w)
    for i in range(w.size):
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd[i] = (mlp.mse(mlp.forward(wp, X, layers)[0], T)
                 - mlp.mse(mlp.forward(wm, X, layers)[0], T)) / (2 * h)
    assert np.abs(g - fd).max() <= 1e-6 * max(1.0, np.abs(fd).max())


def test_silu_and_derivative_match_torch():
    z = np.linspace(-30, 30, 601)
    zt = torch.tensor(z, requires_grad=True)
    s = torch.nn.functional.silu(zt)
    s.sum().backward()
    assert np.allclose(mlp.silu(z), s.detach().numpy(), rtol=1e-14, atol=1e-300)
    assert np.allclose(mlp.dsilu(z), zt.grad.numpy(), rtol=1e-13, atol=1e-15)


def test_adam_matches_torch_optimizer():
    rng = np.random.default_rng(5)
    w = rng.normal(size=50)
    m = np.zeros(50)
    v = np.zeros(50)
    wt = torch.tensor(w.copy(), requires_grad=True)
    opt = torch.optim.Adam([wt], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    for t in range(1, 8):
        g = rng.normal(size=50) * 10.0 ** rng.uniform(-4, 1)
        mlp.adam(w, g, m, v, t, 3e-3)
        wt.grad = torch.tensor(g)
        opt.step()
    assert np.allclose(w, wt.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_occupancy_equals_c_voxelization_at_32():
    """With a 32^3 box the 32^3 sample points are the lattice nodes, so the
    pooled occupancy is the solid fraction of the C oracle's node classes."""
    S = synth.tetra_throat((15.5, 15.5, 15.5), 24.0, (9.0, 10.5, 8.0, 9.5))
    p = synth.Problem(nx=32, ny=32, nz=32, spheres=S, prism_ids=(0, 1, 2), probe=None)
    t = oracle.Oracle(p).types().reshape(32, 32, 32)
    solid = (t == oracle.SOLID).astype(float)
    occ = solid.reshape(4, 8, 4, 8, 4, 8).mean(axis=(1, 3, 5)).ravel()
    d = mlp.descriptor(S, 32, 32, 32)
    assert np.array_equal(d[16:], occ)
    assert 0.0 < occ.mean() < 1.0


def test_occupancy_closed_forms():
    far = [[1e6, 1e6, 1e6, 1e-3]]
    # a triangle enclosing the whole box and four far-away dust spheres: empty
    S = np.array([[-500.0, -500.0, 0, 1e-3], [1500.0, -500.0, 0, 1e-3], [0.0, 1500.0, 0, 1e-3]] + far)
    d = mlp.descriptor(S, 40, 24, 56)
    assert np.all(d[16:] == 0.0)
    # one sphere swallowing the box: full
    S2 = S.copy()
    S2[3] = [20.0, 12.0, 28.0, 1e3]
    assert np.all(mlp.descriptor(S2, 40, 24, 56)[16:] == 1.0)
    # an edge of the triangle on the plane x = 19.5 of a 40-wide box: the
    # samples at x < 19.5 (first two pooled cells in x) are outside
    S3 = np.array([[19.5, -500.0, 0, 1e-3], [19.5, 1500.0, 0, 1e-3], [3000.0, 500.0, 0, 1e-3]] + far)
    occ = mlp.descriptor(S3, 40, 24, 56)[16:].reshape(4, 4, 4)
    assert np.all(occ[:, :, :2] == 1.0) and np.all(occ[:, :, 2:] == 0.0)


def test_geometry_features_invariances():
    S = synth.tetra_throat((24.5, 24.5, 24.5), 24.0, (9.0, 10.5, 8.0, 9.5))
    d = mlp.descriptor(S, 50, 50, 50)[:16]
    assert abs(d[:3].mean() - 1.0) < 1e-15
    assert np.allclose(d[4:13].reshape(3, 3).mean(axis=0), 0.0, atol=1e-14)
    # translating and scaling the spheres leaves the 16 geometry values alone
    S2 = S.copy()
    S2[:, :3] = S2[:, :3] * 1.7 + np.array([3.0, -2.0, 5.0])
    S2[:, 3] *= 1.7
    assert np.allclose(mlp.descriptor(S2, 90, 90, 90)[:16], d, rtol=1e-12, atol=1e-12)


def test_training_reduces_loss_and_ensemble_fallback():
    rng = np.random.default_rng(7)
    layers = mlp.LAYERS
    X = rng.normal(size=(96, 80))
    T = np.tanh(X[:, :17] + 0.5 * X[:, 17:34])
    members = [_rand_member(layers, 10 + z, 0.05) for z in range(2)]
    order = np.stack([np.stack([rng.permutation(96) for _ in range(2)]) for _ in range(6)])
    xs, ts, hist = mlp.train(members, X, T, order, batch=32, lr_max=2e-3, epochs=6)
    assert hist[-1] < 0.6 * hist[0]
    mean, std = mlp.predict(members, xs, ts, X[:5])
    assert mean.shape == (5, 17) and np.all(std >= 0)
    # identical members never fall back; a planted disagreement does
    same = [members[0], members[0].copy()]
    m0, s0 = mlp.predict(same, xs, ts, X[:5])
    assert np.all(s0 == 0) and not mlp.fallback(m0, s0, 0.02).any()
    far = members[0].copy()
    far[-17] += 50.0      # output-0 bias of member 1 only
    m1, s1 = mlp.predict([members[0], far], xs, ts, X[:5])
    assert mlp.fallback(m1, s1, 0.02).all()


def test_opening_radius_closed_form_and_geometry():
    # three equal touching circles: the gap circle has radius R (2/sqrt(3) - 1)
    R = 5.0
    tri = np.array([[0.0, 0.0], [2 * R, 0.0], [R, R * np.sqrt(3.0)]])
    S = np.column_stack([tri, np.zeros(3), np.full(3, R)])
    assert abs(mlp.opening_radius(S) - R * (2 / np.sqrt(3.0) - 1)) < 1e-10
    # unequal radii: the circle is tangent to all three, from outside
    S2 = np.array([[3.0, 1.0, 0.0, 4.0], [15.0, 2.0, 0.0, 6.0], [8.0, 13.0, 0.0, 5.0]])
    r = mlp.opening_radius(S2)
    from scipy.optimize import minimize
    c = minimize(lambda v: sum((np.hypot(v[0] - s[0], v[1] - s[1]) - r - s[3]) ** 2 for s in S2),
                 S2[:, :2].mean(0), tol=1e-14).x
    assert max(abs(np.hypot(c[0] - s[0], c[1] - s[1]) - r - s[3]) for s in S2) < 1e-6
    assert r > 0
