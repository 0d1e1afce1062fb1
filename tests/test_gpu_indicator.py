"""GPU tests of the learned smoothness indicator (through the C ABI).

Features, labels and the network's logits are compared with the FP64 oracle on the same seeded
inputs; the trainer's gradient with the oracle's back-propagation; training must lower the loss
and be deterministic; and the "gain" case checks that a trained indicator skips a large part of a
dam break while the mixed-precision run stays within the benchmark's error bound of the oracle.
"""
import numpy as np
import pytest

import oracle as o
import workloads as w

pytestmark = pytest.mark.gpu

TOL_FP32_REL_L1 = 1e-5   # relative L1 error bound of the FP32 path against the FP64 oracle
LABEL_TOL = 1e-7         # label: nonlinear and linear reconstruction agree to 1e-7 x scale
# bf16 operands: each rounding is within 2^-9 relative; a product of two rounded operands within
# about 2^-8, and the hidden activations are rounded once more.  The logit error is then bounded
# by a few 2^-8 of the network evaluated with absolute values (weights, biases, inputs); 2^-6
# leaves a margin over that estimate.
BF16_REL = 2.0 ** -6


@pytest.fixture(scope="module")
def gks():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2306_04467_amd as g

    g.load()
    return g


def _unpack(P):
    n1, h = o.MLP_IN * o.MLP_H, o.MLP_H
    W1 = P[:n1].reshape(o.MLP_IN, h)
    b1 = P[n1:n1 + h]
    W2 = P[n1 + h:n1 + h + h * h].reshape(h, h)
    b2 = P[n1 + h + h * h:n1 + 2 * h + h * h]
    w3 = P[n1 + 2 * h + h * h:n1 + 3 * h + h * h]
    return W1, b1, W2, b2, w3, P[-1]


def _random_params(seed):
    """He-style initialisation: hidden pre-activations of order one for order-one features."""
    rng = np.random.default_rng(seed)
    P = np.zeros(o.MLP_PARAMS)
    W1, b1, W2, b2, w3, _ = _unpack(P)
    W1[:] = rng.normal(0, np.sqrt(2.0 / o.MLP_IN), W1.shape)
    b1[:] = rng.normal(0, 0.1, b1.shape)
    W2[:] = rng.normal(0, np.sqrt(2.0 / o.MLP_H), W2.shape)
    b2[:] = rng.normal(0, 0.1, b2.shape)
    w3[:] = rng.normal(0, np.sqrt(1.0 / o.MLP_H), w3.shape)
    P[-1] = 0.1
    return P.astype(np.float32)


def _abs_network(P, X):
    """The network with every weight, bias and input replaced by its magnitude and no ReLU:
    an upper bound of the size of every partial sum (for the bf16 error bound)."""
    W1, b1, W2, b2, w3, b3 = (np.abs(a) for a in _unpack(P.astype(np.float64)))
    a1 = np.abs(X) @ W1 + b1
    a2 = a1 @ W2 + b2
    return a2 @ w3 + b3


CASES = {
    "dam_break": lambda: w.dam_break(12),
    "lake_perturbed": lambda: w.lake_at_rest(12, perturb=1e-2, seed=5),
    "smooth_periodic": lambda: w.smooth_periodic(10),
}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_features_match_oracle(gks, case, precision):
    sc = CASES[case]()
    st = gks.State.from_scenario(gks.Mesh.from_scenario(sc), sc, precision=precision)
    X = st.features().astype(np.float64)
    Xr = o.features(o.Mesh.from_scenario(sc), sc.W0, sc.gradW0)
    # FP64 state: the features are computed in double and rounded to float once; FP32 state: the
    # stored gradients carry float rounding as well
    rel = 1e-6 if precision == "fp64" else 1e-5
    tol = rel * (1.0 + np.abs(Xr)) + _flat_stencil_slack(sc, Xr)
    bad = np.abs(X - Xr) > tol
    assert not bad.any(), (case, precision, np.argwhere(bad)[:5], np.abs(X - Xr)[bad][:5], tol[bad][:5])


def _flat_stencil_slack(sc, Xr):
    """Extra tolerance where a field's stencil is flat or nearly so.  There s = max |Q_l - Q_0| +
    1e-12 |Q_0| is tiny, and the features magnify the last bits of the inputs: eta1 = h1 + B and
    grad(eta1) = grad(h1) + grad(B), where each side averages the piecewise-linear bottom and takes
    its gradient itself (rounding differences of a few ulps)."""
    a = 0.5 * np.abs(np.cross(np.c_[sc.node_xy[sc.tri[:, 1]] - sc.node_xy[sc.tri[:, 0]], np.zeros(sc.n_tri)],
                              np.c_[sc.node_xy[sc.tri[:, 2]] - sc.node_xy[sc.tri[:, 0]], np.zeros(sc.n_tri)])[:, 2])
    hs = np.sqrt(2 * a)
    xy, B = sc.node_xy[sc.tri], sc.node_B[sc.tri]
    J = np.stack([xy[:, 1] - xy[:, 0], xy[:, 2] - xy[:, 0]], axis=1)       # rows: edge vectors
    gB = np.abs(np.linalg.solve(J, np.stack([B[:, 1] - B[:, 0], B[:, 2] - B[:, 0]], axis=1)[:, :, None])).max()
    om = o.Mesh.from_scenario(sc)
    slack = np.zeros_like(Xr)
    for f, Q in ((0, sc.W0[3] + B.mean(axis=1)), (1, sc.W0[0])):
        q_eps = 8 * 2.0 ** -52 * np.abs(Q).max()
        g_eps = 64 * 2.0 ** -52 * gB
        for c in range(sc.n_tri):
            cells, _ = om.stencil(c)
            s = np.abs(Q[cells[1:]] - Q[c]).max() + 1e-12 * abs(Q[c])
            x = Xr[c, 17 * f:17 * f + 17]
            slack[c, 17 * f:17 * f + 17] = (1 + np.abs(x)) * q_eps / s
            slack[c, 17 * f + 9:17 * f + 17] += hs[c] * g_eps / s
            slack[c, 34 + f] = q_eps / s        # log10(s / h) / 4
    return slack


def _oracle_labels(sc, tol, G=9.81):
    """(label, ratio): ratio = max over components and Gauss points of |nonlinear - linear| /
    (tol x scale); label = ratio <= 1."""
    om = o.Mesh.from_scenario(sc)
    W, gW = sc.W0, sc.gradW0
    ratio = np.zeros(sc.n_tri)
    for c in range(sc.n_tri):
        vn, _, _ = om.reconstruct(c, W, gW, linear=False)
        vl, _, _ = om.reconstruct(c, W, gW, linear=True)
        h2, h1 = W[0, c], W[3, c]
        scale = np.array([h2, h2 * np.sqrt(G * h2), h2 * np.sqrt(G * h2),
                          h1, h1 * np.sqrt(G * h1), h1 * np.sqrt(G * h1)])
        ratio[c] = (np.abs(vn - vl) / (tol * scale)[None, :]).max()
    return (ratio <= 1.0).astype(np.uint8), ratio


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("tol", [LABEL_TOL, 1e-4])
def test_labels_match_oracle(gks, case, tol):
    sc = CASES[case]()
    st = gks.State.from_scenario(gks.Mesh.from_scenario(sc), sc, precision="fp64")
    y = st.labels(tol)
    yr, ratio = _oracle_labels(sc, tol)
    # the decision is taken in FP64 on both sides from reconstructions that agree to ~1e-15 of
    # the scale; only cells within 1e-6 of the decision boundary may differ
    clear = np.abs(ratio - 1.0) > 1e-6
    assert (y[clear] == yr[clear]).all(), (case, np.flatnonzero((y != yr) & clear)[:10])
    assert set(np.unique(y)) <= {0, 1}


@pytest.mark.parametrize("case", sorted(CASES))
def test_indicator_logits_and_mask(gks, case):
    sc = CASES[case]()
    st = gks.State.from_scenario(gks.Mesh.from_scenario(sc), sc, precision="fp64")
    P = _random_params(11)
    Xr = o.features(o.Mesh.from_scenario(sc), sc.W0, sc.gradW0)
    zr = o.mlp_forward(P.astype(np.float64), Xr)
    thr = float(np.median(zr))
    st.indicator(P, thr)
    z, mask, n_skip = st.indicator_eval()
    # against the FP64 network on the oracle's features: within the bf16 error bound
    bound = BF16_REL * _abs_network(P, Xr)
    assert (np.abs(z - zr) <= bound).all(), (np.abs(z - zr) / bound).max()
    # the fused kernel is the network applied to the state's own features, bit for bit
    X = st.features()
    tr = gks.Trainer(sc.n_tri, P, max_batch=64)
    tr.add(X, np.zeros(sc.n_tri, dtype=np.uint8))
    assert np.array_equal(tr.logits(), z)
    assert np.array_equal(mask, (z > np.float32(thr)).astype(np.uint8))
    assert n_skip == int(mask.sum())


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_fused_indicator_matches_standalone_evaluation(gks, precision):
    """The reconstruction kernel's fused indicator takes, for every cell, the decision of the
    stand-alone network evaluation on the same state (same features, same arithmetic)."""
    sc = w.dam_break(20, bump_amp=0.2)
    m = gks.Mesh.from_scenario(sc)
    st = gks.State.from_scenario(m, sc, precision=precision)
    st.step(3)
    P = _random_params(17)
    st.indicator(P, 0.0)
    z, _, _ = st.indicator_eval()
    thr = float(np.median(z))
    st.indicator(P, thr)
    _, mask, _ = st.indicator_eval()
    st.stage(0)
    fused = st.buffer("skip")[0]
    assert np.array_equal(fused, mask)
    assert 0 < mask.sum() < sc.n_tri


def test_network_inference_matches_bf16_oracle(gks):
    """The matrix-core inference against the oracle's forward pass with the same bf16 operand
    rounding, on identical float inputs (1000 rows: 31 full 32-row tiles and a ragged one)."""
    rng = np.random.default_rng(31)
    N = 1000
    X = (rng.normal(0, 1, (N, o.MLP_IN)) * rng.choice([1e-3, 1.0, 30.0], (N, 1))).astype(np.float32)
    P = _random_params(32)
    tr = gks.Trainer(N, P, max_batch=64)
    tr.add(X, np.zeros(N, dtype=np.uint8))
    z = tr.logits().astype(np.float64)
    zb = o.mlp_forward_bf16(P.astype(np.float64), X.astype(np.float64))
    # same operands on both sides; only the float accumulation order differs (64-term sums)
    tol = 2.0 ** -16 * _abs_network(P, X)
    assert (np.abs(z - zb) <= tol).all(), (np.abs(z - zb) / tol).max()
    for thr in np.quantile(zb, [0.1, 0.5, 0.9]):
        clear = np.abs(zb - thr) > tol
        assert clear.mean() > 0.9
        assert np.array_equal(z[clear] > thr, zb[clear] > thr)


def test_indicator_tail_block(gks):
    """A cell count that is not a multiple of the 32-cell wave tile (ragged last tile)."""
    sc = w.lake_at_rest(7, perturb=1e-2, seed=9)          # 98 cells
    assert sc.n_tri % 32 != 0
    st = gks.State.from_scenario(gks.Mesh.from_scenario(sc), sc, precision="fp32")
    P = _random_params(12)
    Xr = o.features(o.Mesh.from_scenario(sc), sc.W0, sc.gradW0)
    zr = o.mlp_forward(P.astype(np.float64), Xr)
    st.indicator(P, 0.0)
    z, _, _ = st.indicator_eval()
    bound = BF16_REL * _abs_network(P, Xr) + 1e-5 * (1 + np.abs(zr))
    assert (np.abs(z - zr) <= bound).all()


def test_trainer_gradient_matches_oracle(gks):
    rng = np.random.default_rng(21)
    N = 700
    X = rng.normal(0, 1, (N, o.MLP_IN)).astype(np.float32)
    y = (rng.uniform(size=N) < 0.4).astype(np.uint8)
    P = _random_params(13)
    tr = gks.Trainer(N, P, max_batch=512)
    tr.add(X, y)
    assert tr.info() == (N, int(y.sum()))
    for B in (1, 97, 300, 512):                      # single sample, ragged, several blocks
        idx = rng.choice(N, B, replace=B > N).astype(np.int32)
        loss, g = tr.grad(idx)
        lr, gr = o.mlp_grad(P.astype(np.float64), X[idx].astype(np.float64), y[idx].astype(np.float64))
        assert abs(loss - lr) <= 1e-5 * max(1.0, abs(lr)), (B, loss, lr)
        # float accumulation over the batch: error small against the largest gradient entry
        assert np.abs(g - gr).max() <= 1e-4 * np.abs(gr).max(), (B, np.abs(g - gr).max(), np.abs(gr).max())
    with pytest.raises(gks.GksError):
        tr.grad(np.array([N], dtype=np.int32))       # index out of range is rejected
    with pytest.raises(gks.GksError):
        tr.grad(np.zeros(513, dtype=np.int32))       # beyond max_batch


def test_trainer_fit_lowers_loss_and_is_deterministic(gks):
    rng = np.random.default_rng(22)
    N = 5000
    X = rng.normal(0, 1, (N, o.MLP_IN)).astype(np.float32)
    u = rng.normal(0, 1, o.MLP_IN)
    y = (X @ u + 0.5 * np.sin(3 * X[:, 0]) > 0).astype(np.uint8)
    P = _random_params(14)
    runs = []
    for _ in range(2):
        tr = gks.Trainer(N, P, max_batch=256)
        tr.add(X, y)
        losses = tr.fit(8, batch=256, lr=3e-3, seed=5)
        runs.append((losses, tr.params(), tr.logits()))
    losses, P1, z = runs[0]
    assert losses[-1] < 0.5 * losses[0], losses
    assert np.array_equal(runs[0][1], runs[1][1])     # same seed, same order: same parameters
    acc = ((z > 0) == (y == 1)).mean()
    assert acc > 0.9, acc
    # the trained logits with the inference arithmetic agree with the oracle's FP64 forward
    zr = o.mlp_forward(P1.astype(np.float64), X.astype(np.float64))
    assert (np.abs(z - zr) <= BF16_REL * _abs_network(P1, X)).all()


def test_trainer_threshold_bounds_false_skips(gks):
    rng = np.random.default_rng(23)
    N = 4000
    X = rng.normal(0, 1, (N, o.MLP_IN)).astype(np.float32)
    y = (X[:, 0] > 0).astype(np.uint8)
    tr = gks.Trainer(N, _random_params(15), max_batch=512)
    tr.add(X, y)
    tr.fit(3, batch=512, lr=3e-3, seed=1)
    z = tr.logits()
    for rate in (0.0, 1e-3, 1e-2):
        thr = tr.threshold(rate)
        false_skips = ((z > thr) & (y == 0)).sum()
        assert false_skips <= int(np.floor(rate * N)), (rate, false_skips)
        # and the threshold is the smallest such: lowering it to the next logit would exceed
        assert ((z >= thr) & (y == 0)).sum() > int(np.floor(rate * N)) or thr == np.float32(-3.4028235e38)


def _rel_l1(W, Wr, area, G=9.81):
    out = []
    for o_ in (0, 3):
        h = Wr[o_]
        out.append((area * np.abs(W[o_] - h)).sum() / (area * np.abs(h)).sum())
        den = (area * h * np.sqrt(G * h)).sum()
        for v in (o_ + 1, o_ + 2):
            out.append((area * np.abs(W[v] - Wr[v])).sum() / den)
    return np.array(out)


def test_indicator_gain_case(gks):
    """Train on FP64 snapshots of dam breaks and perturbed lakes, then run an unseen dam break in
    FP32 with and without the indicator for 20 steps: the indicator must skip a large share of the
    cells and both runs must stay within the FP32 error bound of the FP64 oracle."""
    P0 = _random_params(16)
    train = [w.dam_break(24, seed=101), w.lake_at_rest(24, perturb=1e-2, seed=102),
             w.dam_break(24, seed=103, left=(0.8, 0.6), right=(0.6, 0.8), bump_amp=0.2)]
    cap = sum(sc.n_tri for sc in train) * 6
    tr = gks.Trainer(cap, P0, max_batch=512)
    for sc in train:
        st = gks.State.from_scenario(gks.Mesh.from_scenario(sc), sc, precision="fp64")
        for k in range(6):
            tr.add_state(st, LABEL_TOL)
            st.step(5)
    n, npos = tr.info()
    assert n == cap and 0 < npos < n
    losses = tr.fit(30, batch=512, lr=2e-3, seed=7)
    assert losses[-1] < losses[0]
    thr = tr.threshold(1e-4)
    P = tr.params()

    sc = w.dam_break(24, seed=104, bump_amp=0.2)
    om = o.Mesh.from_scenario(sc)
    p = o.params_of(sc)
    a, _, _ = om.geometry()
    m = gks.Mesh.from_scenario(sc)
    full = gks.State.from_scenario(m, sc, precision="fp32")
    ind = gks.State.from_scenario(m, sc, precision="fp32")
    ind.indicator(P, thr)
    W, gW = sc.W0.copy(), sc.gradW0.copy()
    skipped = []
    for _ in range(20):
        dt = o.dt(om, p, W)
        for st in (full, ind):
            st.stage(0, dt)
            st.stage(1)
        _, mask, k = ind.indicator_eval()
        skipped.append(k / sc.n_tri)
        W, gW = o.step(om, p, dt, W, gW)
    Wf, _, _ = full.read()
    Wi, _, _ = ind.read()
    ef, ei = _rel_l1(Wf, W, a).max(), _rel_l1(Wi, W, a).max()
    assert ef <= TOL_FP32_REL_L1, ef
    assert ei <= TOL_FP32_REL_L1, (ei, ef)
    assert np.mean(skipped) > 0.3, skipped


def test_indicator_at_full_size(gks):
    """The gain workload at its full size (2,000,000 triangles, dam break over a bump, FP32): a
    network trained as in the gain case above, fused into the reconstruction (its first stage
    infers, the second reuses the decisions), for one step with the oracle's step size; with and
    without it the state stays within the FP32 bound of the FP64 oracle's step, and the network
    skips most cells."""
    P0 = _random_params(21)
    train = [w.dam_break(24, seed=111), w.lake_at_rest(24, perturb=1e-2, seed=112),
             w.dam_break(24, seed=113, left=(0.8, 0.6), right=(0.6, 0.8), bump_amp=0.2)]
    tr = gks.Trainer(sum(sc.n_tri for sc in train) * 6, P0, max_batch=512)
    for sc in train:
        st = gks.State.from_scenario(gks.Mesh.from_scenario(sc), sc, precision="fp64")
        for k in range(6):
            tr.add_state(st, LABEL_TOL)
            st.step(5)
    tr.fit(30, batch=512, lr=2e-3, seed=7)
    thr, P = tr.threshold(1e-4), tr.params()

    sc = w.dam_break(1000, seed=20230608, sin_amp=0.1, bump_amp=0.2)
    print(f"[indicator] full size T={sc.n_tri}", flush=True)
    om = o.Mesh.from_scenario(sc)
    p = o.params_of(sc)
    a, _, _ = om.geometry()
    m = gks.Mesh.from_scenario(sc)
    full = gks.State.from_scenario(m, sc, precision="fp32")
    ind = gks.State.from_scenario(m, sc, precision="fp32")
    ind.indicator(P, thr)
    dt = o.dt(om, p, sc.W0)
    for st in (full, ind):
        st.stage(0, dt)
        st.stage(1)
    W, _ = o.step(om, p, dt, sc.W0, sc.gradW0)
    _, _, k = ind.indicator_eval()
    ef = _rel_l1(full.read()[0], W, a).max()
    ei = _rel_l1(ind.read()[0], W, a).max()
    print(f"   rel-L1 full {ef:.2e} indicator {ei:.2e} skipped {k / sc.n_tri:.3f}", flush=True)
    assert ef <= TOL_FP32_REL_L1 and ei <= TOL_FP32_REL_L1, (ef, ei)
    assert k > 0.5 * sc.n_tri
