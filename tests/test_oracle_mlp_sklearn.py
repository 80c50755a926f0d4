"""The FP64 oracle network's training pinned against scikit-learn's
MLPRegressor, the library of the paper's runtime model (Sec. "Hyperparameters",
Table para-setting: Adam, alpha, batch 200, 200 epochs, tol, the stability
factor).

Both are started from the same weights (``inputs.mlp_init``) and visit the
rows in order (``shuffle=False`` there, identity permutations here), so the
two must agree to rounding: epoch losses, final weights, and the epoch at
which the improvement-tolerance rule stops training. scikit-learn is an
independent implementation of the loss, its L2 term, Adam's bias-corrected
step and the stopping rule, so a dropped term, a transposed weight or an
off-by-one in the stop count in the oracle fails here.
"""
import warnings

import numpy as np
import pytest

import oracle.mlp as mlp
from paper_2306_14011_amd import inputs

sklearn = pytest.importorskip("sklearn")


def _data(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, 14))
    y = np.sin(X[:, 0]) + 0.3 * X[:, 1] * X[:, 2] - 0.2 * np.abs(X[:, 5])
    return X, y


def _sklearn_train(theta0, X, y, batch, epochs, tol):
    from sklearn.exceptions import ConvergenceWarning
    from sklearn.neural_network import MLPRegressor
    r = MLPRegressor(hidden_layer_sizes=(64, 64, 64), activation="relu", solver="adam", alpha=1e-4,
                     batch_size=batch, learning_rate="constant", learning_rate_init=9e-4, max_iter=1,
                     shuffle=False, tol=tol, beta_1=0.95, beta_2=0.90, epsilon=1e-9, n_iter_no_change=10,
                     warm_start=True, early_stopping=False, random_state=0)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", ConvergenceWarning)
        warnings.simplefilter("ignore", UserWarning)
        r.fit(X[:5], y[:5])          # builds the layers; the weights are replaced next
    p = mlp.unpack(np.asarray(theta0, dtype=np.float64))
    # scikit-learn stores W[in][out]; the oracle W[out][in]
    r.coefs_ = [p[k].T.copy() for k in ("W1", "W2", "W3", "W4")]
    r.intercepts_ = [p[k].copy() for k in ("b1", "b2", "b3", "b4")]
    r.loss_curve_ = []
    r._no_improvement_count = 0
    r.best_loss_ = np.inf
    r.t_ = 0
    r.n_iter_ = 0
    r.max_iter = epochs
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", ConvergenceWarning)
        r.fit(X, y)
    theta = np.concatenate([np.concatenate([W.T.ravel(), b]) for W, b in zip(r.coefs_, r.intercepts_)])
    return theta, np.array(r.loss_curve_), r.n_iter_


@pytest.mark.parametrize("n,batch,epochs", [(450, 200, 60), (120, 120, 80)], ids=["minibatch_ragged", "full_batch"])
def test_training_matches_sklearn(n, batch, epochs):
    X, y = _data(n, 4)
    theta0 = inputs.mlp_init(3)
    ref, ref_loss, ref_epochs = _sklearn_train(theta0, X, y, batch, epochs, tol=1e-12)
    order = np.tile(np.arange(n, dtype=np.int32), (epochs, 1))
    th, loss, ep, _, _, t = mlp.train(theta0, X, y, order, batch=batch, max_epochs=epochs, tol=1e-12)
    assert ep == ref_epochs == epochs
    assert t == epochs * -(-n // batch)          # one Adam step per minibatch
    assert np.allclose(loss, ref_loss, rtol=1e-12, atol=0), np.abs(loss / ref_loss - 1).max()
    assert np.allclose(th, ref, rtol=0, atol=1e-12 * np.abs(ref).max()), np.abs(th - ref).max()
    assert loss[-1] < 0.5 * loss[0]              # it did learn


def test_early_stop_epoch_matches_sklearn():
    # a coarse tolerance makes the improvement rule end training early; both
    # must stop at the same epoch with the same losses
    X, y = _data(300, 8)
    theta0 = inputs.mlp_init(5)
    ref, ref_loss, ref_epochs = _sklearn_train(theta0, X, y, 200, 200, tol=5e-3)
    order = np.tile(np.arange(300, dtype=np.int32), (200, 1))
    th, loss, ep, _, _, _ = mlp.train(theta0, X, y, order, batch=200, max_epochs=200, tol=5e-3)
    assert 11 < ep < 200
    assert ep == ref_epochs
    assert np.allclose(loss, ref_loss, rtol=1e-12, atol=0)
    assert np.allclose(th, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
