"""Selector network kernels (forward, backward, Adam) against the float64
oracle, and the selector inside plan creation."""
import numpy as np
import pytest

import crsgen
import oracle
from oracle import mlp

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
import paper_1101_0091_amd as pkg  # noqa: E402

DEV = "cuda:0"
U32 = 2.0 ** -24


def _theta32(seed):
    rng = np.random.default_rng(seed)
    parts = [rng.uniform(-0.4, 0.4, size=s) for s in mlp.SHAPES]
    return mlp.pack(parts).astype(np.float32)


def _inputs(nb, seed):
    """Dyadic theta (k/16, |k| <= 4), X (m/2, |m| <= 8) and T (k/16): every
    forward product and partial sum is a multiple of 2^-13 below 2^11, so the
    float32 forward is exact in any summation order and equals the float64
    oracle bit for bit (the ReLU masks then agree as well)."""
    for s in range(seed, seed + 200):
        rng = np.random.default_rng(s)
        th = (rng.integers(-4, 5, size=mlp.N_PARAMS) / 16.0).astype(np.float32)
        X = (rng.integers(-8, 9, size=(nb, 16)) / 2.0).astype(np.float32)
        T = (rng.integers(-64, 65, size=(nb, 7)) / 16.0).astype(np.float32)
        T[::2, 6] = np.nan  # V6 without a time on every other sample
        Yabs, (_, m1, _, m2, _) = mlp.forward(np.abs(th.astype(np.float64)),
                                              np.abs(X.astype(np.float64)))
        if m1.max() < 2.0**19 and m2.max() < 2.0**15 and Yabs.max() < 2.0**10:
            return th, X, T
    raise RuntimeError("no exactly representable inputs")


def _abs_backward(th, cache, dYabs):
    """Backward pass on magnitudes: sum of |terms| of every gradient entry."""
    W1, b1, W2, b2, W3, b3 = mlp.unpack(np.abs(th))
    X, z1, h1, z2, h2 = cache
    X, h1, h2 = np.abs(X), np.abs(h1), np.abs(h2)
    dz2 = (dYabs @ W3) * (z2 > 0)
    dz1 = (dz2 @ W2) * (z1 > 0)
    return mlp.pack([dz1.T @ X, dz1.sum(0), dz2.T @ h1, dz2.sum(0), dYabs.T @ h2,
                     dYabs.sum(0)])


def _run_forward(th, X):
    nb = X.shape[0]
    thd = torch.from_numpy(th).to(DEV)
    Xd = torch.from_numpy(X).to(DEV)
    Y = torch.empty((nb, 7), dtype=torch.float32, device=DEV)
    Z1 = torch.empty((nb, 64), dtype=torch.float32, device=DEV)
    Z2 = torch.empty((nb, 64), dtype=torch.float32, device=DEV)
    pkg.spmv_mlp_forward(thd, Xd, nb, Y, Z1, Z2)
    return thd, Xd, Y, Z1, Z2


@pytest.mark.parametrize("nb", [1, 37, 384])
def test_forward_and_backward_vs_oracle(nb):
    th, X, T = _inputs(nb, 11 + nb)
    th64, X64, T64 = th.astype(np.float64), X.astype(np.float64), T.astype(np.float64)
    thd, Xd, Y, Z1, Z2 = _run_forward(th, X)
    Yref, cache = mlp.forward(th64, X64)
    assert np.array_equal(Y.cpu().numpy(), Yref)
    assert np.array_equal(Z1.cpu().numpy(), cache[1])
    assert np.array_equal(Z2.cpu().numpy(), cache[3])
    Td = torch.from_numpy(T).to(DEV)
    scratch = torch.empty(nb * (7 + 64 + 64), dtype=torch.float32, device=DEV)
    grad = torch.empty(mlp.N_PARAMS, dtype=torch.float32, device=DEV)
    pkg.spmv_mlp_backward(thd, Xd, Z1, Z2, Y, Td, nb, scratch, grad)
    gref = mlp.backward(th64, cache, Yref, T64)
    dYabs = np.where(np.isnan(T64), 0.0, 2.0 * np.abs(Yref - T64) / (nb * 7))
    gabs = _abs_backward(th64, cache, dYabs)
    err = np.abs(grad.cpu().numpy() - gref)
    assert np.all(err <= 1e-4 * gabs + 1e-30), float(np.max(err / (gabs + 1e-30)))


def test_adam_step_vs_oracle():
    rng = np.random.default_rng(3)
    n = mlp.N_PARAMS
    th = rng.standard_normal(n).astype(np.float32)
    g = rng.standard_normal(n).astype(np.float32)
    m = (0.1 * rng.standard_normal(n)).astype(np.float32)
    v = np.abs(0.1 * rng.standard_normal(n)).astype(np.float32)
    d = [torch.from_numpy(a.copy()).to(DEV) for a in (th, g, m, v)]
    pkg.spmv_mlp_adam(d[0], d[1], d[2], d[3], 7, 1e-2, 0.9, 0.999, 1e-8)
    # the kernel receives float32 hyperparameters; the oracle takes the same values
    b1, b2, lr, eps = (float(np.float32(x)) for x in (0.9, 0.999, 1e-2, 1e-8))
    th2, m2, v2 = mlp.adam_step(th.astype(np.float64), g.astype(np.float64),
                                m.astype(np.float64), v.astype(np.float64), 7, lr=lr,
                                beta1=b1, beta2=b2, eps=eps)
    assert np.allclose(d[2].cpu().numpy(), m2, rtol=1e-6, atol=1e-7)
    assert np.allclose(d[3].cpu().numpy(), v2, rtol=1e-6, atol=1e-9)
    assert np.all(np.abs(d[0].cpu().numpy() - th2) <= 1e-6 * np.abs(th2) + 1e-5 * 1e-2)


def test_training_reduces_loss():
    """A few hundred Adam steps on a learnable target lower the loss."""
    nb = 256
    rng = np.random.default_rng(9)
    X = rng.standard_normal((nb, 16)).astype(np.float32)
    Wt = rng.standard_normal((16, 7)) / 4
    T = np.tanh(X.astype(np.float64) @ Wt).astype(np.float32)
    th = _theta32(5) * 0.5
    thd = torch.from_numpy(th).to(DEV)
    Xd, Td = torch.from_numpy(X).to(DEV), torch.from_numpy(T).to(DEV)
    Y = torch.empty((nb, 7), dtype=torch.float32, device=DEV)
    Z1 = torch.empty((nb, 64), dtype=torch.float32, device=DEV)
    Z2 = torch.empty((nb, 64), dtype=torch.float32, device=DEV)
    sc = torch.empty(nb * 135, dtype=torch.float32, device=DEV)
    g = torch.empty(mlp.N_PARAMS, dtype=torch.float32, device=DEV)
    m = torch.zeros_like(g)
    v = torch.zeros_like(g)
    losses = []
    for t in range(1, 301):
        pkg.spmv_mlp_forward(thd, Xd, nb, Y, Z1, Z2)
        if t in (1, 300):
            losses.append(float(((Y - Td) ** 2).mean()))
        pkg.spmv_mlp_backward(thd, Xd, Z1, Z2, Y, Td, nb, sc, g)
        pkg.spmv_mlp_adam(thd, g, m, v, t, 3e-3)
    assert losses[1] < 0.3 * losses[0], losses


def test_selector_in_create_matches_oracle_forward():
    th = _theta32(21)
    mu = np.linspace(-1, 1, 16).astype(np.float32)
    sigma = np.linspace(0.5, 3, 16).astype(np.float32)
    lo = np.full(16, -1e30, np.float32)
    hi = np.full(16, 1e30, np.float32)
    pkg.spmv_selector_load(th, mu, sigma, lo, hi, 0.0)
    assert pkg.spmv_selector_loaded()
    A = crsgen.mesh3d(30, seed=3)[0]
    M = pkg.CRSMatrix.from_crs(A, device=DEV)  # default mode runs the selector
    pred = pkg.spmv_get_predictions(M.handle)
    f = oracle.row_features(A.n_rows, A.row_ptr, A.col_idx)
    x = ((f.astype(np.float32) - mu) / sigma).astype(np.float64)
    yref, _ = mlp.forward(th.astype(np.float64), x[None, :])
    yabs, _ = mlp.forward(np.abs(th.astype(np.float64)), np.abs(x[None, :]))
    assert np.all(np.abs(pred - yref[0]) <= 1e-4 * yabs[0] + 1e-6)
    # no V6 copy: the V6 output is not a candidate
    assert M.variant == int(np.argmin(pred[:6]))
    # with the copy (a matrix whose chunks fit the reserve) every output is
    L = crsgen.laplace2d(96)
    for fl in (0, pkg.SPMV_FLAG_SELL):
        ML = pkg.CRSMatrix.from_crs(L, flags=fl, device=DEV)
        pl = pkg.spmv_get_predictions(ML.handle)
        assert (ML.sell_slots is not None) == bool(fl)
        assert ML.variant == int(np.argmin(pl if fl else pl[:6]))
    # MLP mode with an unreachable margin falls back to autotune
    pkg.spmv_selector_load(th, mu, sigma, lo, hi, 1e9)
    M2 = pkg.CRSMatrix.from_crs(A, flags=pkg.SPMV_SELECT_MLP, device=DEV)
    t = pkg.spmv_get_autotune_times(M2.handle)
    assert M2.variant == int(np.argmin(t))


def test_packaged_selector_choice_matches_oracle():
    """With the trained weights, plan creation picks argmin of the network
    output; the oracle network on the oracle features picks the same variant
    unless its best two outputs are within float32 noise."""
    import os
    from paper_1101_0091_amd.selector import DEFAULT_WEIGHTS, unpack_weights
    if not os.path.exists(DEFAULT_WEIGHTS):
        pytest.skip("no trained weights")
    pkg.load_selector(DEFAULT_WEIGHTS)
    theta, mu, sigma, lo, hi, margin = unpack_weights(DEFAULT_WEIGHTS)
    agree = 0
    for idx in range(12):
        A, _ = crsgen.family_matrix(9, idx, 2e3, 3e5)
        M = pkg.CRSMatrix.from_crs(A, device=DEV)  # no V6 copy: outputs V0-V5
        f = oracle.row_features(A.n_rows, A.row_ptr, A.col_idx)
        x = ((f.astype(np.float32) - mu) / sigma).astype(np.float64)
        y = mlp.forward(theta.astype(np.float64), x[None, :])[0][0][:6]
        srt = np.sort(y)
        if srt[1] - srt[0] > 1e-3:
            assert M.variant == int(np.argmin(y)), (idx, M.variant, y)
            agree += 1
    assert agree >= 6
