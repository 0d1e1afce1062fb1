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
    assert X.shape == (sc.n_tri, o.MLP_IN) and np.isfinite(X).all()
    # thickness features depend on differences only, normalised by their largest magnitude, and
    # the size features compare that magnitude with the thickness: h -> 3 h changes none of them
    # beyond the 1e-12 |Q0| floor; at rest the momentum features sit at the floor, log10(1e-12)/4
    W, gW = sc.W0.copy(), sc.gradW0.copy()
    W[[0, 3]] *= 3.0
    gW[[0, 3]] *= 3.0
    X3 = o.features(m, W, gW)
    nz = np.abs(X[:, :34]).max(axis=1) > 1e-3
    np.testing.assert_allclose(X3[nz, :36], X[nz, :36], rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(X[:, 36:38], -3.0, rtol=0, atol=1e-12)
    np.testing.assert_allclose(X3[:, 36:38], -3.0, rtol=0, atol=1e-12)
    # a flat h2 stencil: s = 1e-12 h2, so the size feature is log10(1e-12)/4
    flat_h2 = (X[:, 17:26] == 0).all(axis=1)
    assert flat_h2.any()
    np.testing.assert_allclose(X[flat_h2, 35], -3.0, rtol=0, atol=1e-12)
    # the size feature of a stencil with variation is log10(max |Q_l - Q_0| / h) / 4
    c = int(np.flatnonzero(nz)[0])
    cells, _ = m.stencil(c)
    s = np.abs(sc.W0[3, cells[1:]] - sc.W0[3, c]).max() + 1e-12 * sc.W0[3, c]
    np.testing.assert_allclose(X[c, 34], np.log10(s / sc.W0[3, c]) / 4, rtol=1e-12)
    # geometry features: area ratios of face neighbours and edge lengths over sqrt(2 |Omega|)
    a, _, _ = m.geometry()
    xy = sc.node_xy[sc.tri]
    lens = np.linalg.norm(np.roll(xy, -1, axis=1) - xy, axis=2)
    np.testing.assert_allclose(X[:, 41:44], lens / np.sqrt(2 * a)[:, None], rtol=1e-13)
    for c in range(0, sc.n_tri, 7):
        cells, _ = m.stencil(c)
        np.testing.assert_allclose(X[c, 38:41], a[cells[1:4]] / a[c], rtol=1e-14)


def test_momentum_features_measure_the_layer_momentum_variation():
    sc = w.lake_at_rest(6, bump_amp=0.0)
    rng = np.random.default_rng(3)
    sc.W0[4] = 1e-3 * rng.normal(size=sc.n_tri)   # lower-layer x-momentum only
    m = o.Mesh.from_scenario(sc)
    X = o.features(m, sc.W0, sc.gradW0, G=9.81)
    np.testing.assert_allclose(X[:, 37], -3.0, rtol=0, atol=1e-12)  # upper layer at rest
    for c in range(0, sc.n_tri, 5):
        cells, maps = m.stencil(c)
        h1 = sc.W0[3, c]
        cm = h1 * np.sqrt(9.81 * h1)
        # images: rotate (h1U1, h1V1) by each map (the identity for interior neighbours)
        mom = np.array([[maps[l, 0] * sc.W0[4, n] + maps[l, 1] * sc.W0[5, n],
                         maps[l, 2] * sc.W0[4, n] + maps[l, 3] * sc.W0[5, n]] for l, n in enumerate(cells)])
        sm = np.abs(mom[1:] - mom[0]).max()
        np.testing.assert_allclose(X[c, 36], np.log10((sm + 1e-12 * cm) / cm) / 4, rtol=1e-12)


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


def test_bf16_forward_equals_fp64_forward_on_representable_operands():
    # small integers are exact in bfloat16 (8 significant bits) and so are the hidden sums here
    rng = np.random.default_rng(7)
    P = np.zeros(o.MLP_PARAMS)
    W1, b1, W2, b2, w3 = _unpack(P)
    W1[:] = rng.integers(-1, 2, W1.shape)
    b1[:] = rng.integers(-1, 2, b1.shape)
    W2[:] = rng.integers(-1, 2, W2.shape)
    b2[:] = rng.integers(-3, 4, b2.shape)
    w3[:] = rng.normal(size=w3.shape)
    P[-1] = -0.3
    X = rng.integers(-2, 3, (9, o.MLP_IN)).astype(float)
    assert np.array_equal(o.mlp_forward_bf16(P, X), o.mlp_forward(P, X))


def test_bf16_forward_rounds_inputs_to_nearest_even():
    # permutation network with unit gains: z = b3 + sum_i w3[perm(i)] relu(bf16(x_i)).  bfloat16
    # has a spacing of 2^-7 on [1, 2): 1 + 2^-8 is a tie and goes to the even 1; 1 + 3 2^-8 is a
    # tie between 1 + 2^-7 (odd) and 1 + 2^-6 (even); anything above a tie rounds up.
    P = np.zeros(o.MLP_PARAMS)
    W1, b1, W2, b2, w3 = _unpack(P)
    perm = np.arange(o.MLP_IN)[::-1]
    W1[np.arange(o.MLP_IN), perm] = 1.0
    W2[:] = np.eye(o.MLP_H)
    w3[:] = 0.0
    cases = [(1 + 2 ** -8, 1.0), (1 + 3 * 2 ** -8, 1 + 2 ** -6), (1 + 2 ** -8 + 2 ** -20, 1 + 2 ** -7),
             (-5.0, 0.0), (3 - 2 ** -9, 3.0), (255.4, 255.0), (257.0, 256.0)]
    for k, (x, r) in enumerate(cases):
        X = np.zeros((1, o.MLP_IN))
        X[0, k] = x
        w3[:] = 0.0
        w3[perm[k]] = 1.0
        assert o.mlp_forward_bf16(P, X)[0] == r, (x, r)
