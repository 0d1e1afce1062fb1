"""Pins of the oracle's smoothness-indicator pieces: the MLP gradient against central finite
differences, and the features' invariance under an affine change of the variables."""
import numpy as np

import oracle as o
import workloads as w


def _params(seed=0):
    rng = np.random.default_rng(seed)
    P = rng.normal(0, 0.3, o.MLP_PARAMS)
    return P


def test_mlp_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    P = _params()
    X = rng.normal(0, 1, (16, o.MLP_IN))
    y = (rng.uniform(size=16) > 0.5).astype(float)
    loss, g = o.mlp_grad(P, X, y)
    z = o.mlp_forward(P, X)
    ref_loss = np.mean(np.logaddexp(0, z) - y * z)
    assert abs(loss - ref_loss) < 1e-13
    idx = rng.choice(o.MLP_PARAMS, 120, replace=False)
    idx = np.concatenate([idx, [o.MLP_PARAMS - 1, 2560, 2560 + 64 + 100]])
    for i in idx:
        h = 1e-6
        Pp, Pm = P.copy(), P.copy()
        Pp[i] += h
        Pm[i] -= h
        fd = (o.mlp_grad(Pp, X, y)[0] - o.mlp_grad(Pm, X, y)[0]) / (2 * h)
        assert abs(fd - g[i]) < 1e-7 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_features_invariant_under_affine_change_of_the_thicknesses():
    sc = w.dam_break(8, sin_amp=0.0, bump_amp=0.0)  # flat bottom: eta1 = h1 scales with h1
    sc.W0[3] += 0.02 * np.sin(7 * sc.node_xy[sc.tri].mean(axis=1)[:, 1])
    m = o.Mesh.from_scenario(sc)
    X = o.features(m, sc.W0, sc.gradW0)
    assert X.shape == (sc.n_tri, 40) and np.isfinite(X).all()
    # thickness features depend on differences only, normalised by their largest magnitude:
    # h -> 3 h changes no thickness feature beyond the 1e-12 |Q0| floor
    W, gW = sc.W0.copy(), sc.gradW0.copy()
    W[[0, 3]] *= 3.0
    gW[[0, 3]] *= 3.0
    X3 = o.features(m, W, gW)
    nz = np.abs(X[:, :34]).max(axis=1) > 1e-3
    np.testing.assert_allclose(X3[nz, :34], X[nz, :34], rtol=1e-9, atol=1e-9)
    # geometry features: area ratios of face neighbours and edge lengths over sqrt(2 |Omega|)
    a, _, _ = m.geometry()
    xy = sc.node_xy[sc.tri]
    lens = np.linalg.norm(np.roll(xy, -1, axis=1) - xy, axis=2)
    np.testing.assert_allclose(X[:, 37:40], lens / np.sqrt(2 * a)[:, None], rtol=1e-13)
    assert (X[:, 34:37] > 0).all()


def _unpack(P):
    n1, h = o.MLP_IN * o.MLP_H, o.MLP_H
    W1 = P[:n1].reshape(o.MLP_IN, h)
    b1 = P[n1:n1 + h]
    W2 = P[n1 + h:n1 + h + h * h].reshape(h, h)
    b2 = P[n1 + h + h * h:n1 + 2 * h + h * h]
    w3 = P[n1 + 2 * h + h * h:n1 + 3 * h + h * h]
    return W1, b1, W2, b2, w3


def test_mlp_forward_on_a_permutation_network():
    # W1 routes input i to hidden unit perm(i) with gain a_i, W2 is the identity, no biases:
    # z = sum_i w3[perm(i)] relu(a_i x_i).  A transposed weight matrix or a swapped layer fails.
    rng = np.random.default_rng(5)
    P = np.zeros(o.MLP_PARAMS)
    W1, b1, W2, b2, w3 = _unpack(P)
    perm = rng.permutation(o.MLP_H)[:o.MLP_IN]
    a = rng.uniform(0.5, 2.0, o.MLP_IN)
    W1[np.arange(o.MLP_IN), perm] = a
    W2[:] = np.eye(o.MLP_H)
    w3[:] = rng.normal(size=o.MLP_H)
    P[-1] = 0.25
    X = rng.normal(size=(7, o.MLP_IN))
    z = o.mlp_forward(P, X)
    expect = 0.25 + (np.maximum(a * X, 0) * w3[perm]).sum(axis=1)
    np.testing.assert_allclose(z, expect, rtol=1e-14, atol=1e-14)


def test_mlp_forward_is_positively_homogeneous_without_biases():
    rng = np.random.default_rng(6)
    P = _params(3)
    W1, b1, W2, b2, w3 = _unpack(P)
    b1[:] = 0
    b2[:] = 0
    P[-1] = 0
    X = rng.normal(size=(5, o.MLP_IN))
    np.testing.assert_allclose(o.mlp_forward(P, 2.5 * X), 2.5 * o.mlp_forward(P, X), rtol=1e-12, atol=1e-14)
