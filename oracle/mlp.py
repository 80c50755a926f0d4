"""FP64 reference of the autotuner's runtime-regression network.

TEST INFRASTRUCTURE (see the package docstring). Follows the paper's
Sec. "Hyperparameters" and Table para-setting: a fully connected ReLU network
regressing runtime on the launch parameters, trained by Adam with an L2
penalty alpha, minibatches of 200, at most 200 epochs, an improvement
tolerance, and a numerical stability factor. Features are standardised
(Sec. "Feature Centering and Scaling": mean removal and unit variance), and
accuracy is R^2 (Eq. R_square).

Conventions (the paper does not print them; scikit-learn's documented ones):
  * loss of a minibatch of B rows: sum (yhat - y)^2 / (2B) + alpha/(2B) * sum W^2,
    biases not penalised;
  * Adam, efficient form of Kingma & Ba: m = b1 m + (1-b1) g,
    v = b2 v + (1-b2) g^2, theta -= lr sqrt(1-b2^t)/(1-b1^t) m/(sqrt(v)+eps);
  * epoch loss = sum over minibatches of L_b * B_b / n; training stops once
    the epoch loss has failed to improve on the best by tol for more than
    n_iter_no_change consecutive epochs;
  * ReLU'(0) = 0.
Parameter layout: W1[64][n_in], b1, W2[64][64], b2, W3[64][64], b3, W4[1][64], b4,
with n_in = 14 for the paper's network (the launch features) and n_in = 16 for
the problem-size-conditioned one (the launch features, then the log2 cell
count and the dimension); n_in follows from the length of theta.
"""
from __future__ import annotations

import numpy as np

IN = 14
IN_SIZED = 16
H = 64


def shapes(n_in=IN):
    return [("W1", (H, n_in)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)),
            ("W3", (H, H)), ("b3", (H,)), ("W4", (1, H)), ("b4", (1,))]


def nparam(n_in=IN):
    return sum(int(np.prod(s)) for _, s in shapes(n_in))


SHAPES = shapes(IN)
NPARAM = nparam(IN)


def n_in_of(theta):
    """Input width of the network whose flat parameters are theta."""
    n_in, rem = divmod(len(theta) - nparam(0), H)
    if rem or n_in < 1:
        raise ValueError("not a parameter vector of this network")
    return n_in


def unpack(theta):
    out = {}
    o = 0
    for name, shp in shapes(n_in_of(theta)):
        k = int(np.prod(shp))
        out[name] = theta[o:o + k].reshape(shp)
        o += k
    return out


def weight_mask(n_in=IN):
    """1 for weights, 0 for biases, in the flat layout."""
    m = []
    for name, shp in shapes(n_in):
        m.append(np.full(int(np.prod(shp)), 1.0 if name.startswith("W") else 0.0))
    return np.concatenate(m)


def relu(z):
    return np.where(z > 0.0, z, 0.0)


def forward(theta, X):
    p = unpack(np.asarray(theta, dtype=np.float64))
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ p["W1"].T + p["b1"]
    z2 = relu(z1) @ p["W2"].T + p["b2"]
    z3 = relu(z2) @ p["W3"].T + p["b3"]
    out = (relu(z3) @ p["W4"].T + p["b4"])[:, 0]
    return out, (X, z1, z2, z3)


def predict(theta, X):
    return forward(theta, X)[0]


def loss_grad(theta, X, y, alpha):
    """Loss of the rows (X, y) and its gradient with respect to theta."""
    theta = np.asarray(theta, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    B = X.shape[0]
    p = unpack(theta)
    out, (X, z1, z2, z3) = forward(theta, X)
    d = out - y
    n_in = n_in_of(theta)
    mask = weight_mask(n_in)
    loss = 0.5 * np.sum(d * d) / B + 0.5 * alpha * np.sum(theta * theta * mask) / B
    dout = d / B
    g = {}
    h3 = relu(z3)
    g["W4"] = dout[None, :] @ h3
    g["b4"] = np.array([dout.sum()])
    d3 = (dout[:, None] * p["W4"]) * (z3 > 0.0)
    h2 = relu(z2)
    g["W3"] = d3.T @ h2
    g["b3"] = d3.sum(axis=0)
    d2 = (d3 @ p["W3"]) * (z2 > 0.0)
    h1 = relu(z1)
    g["W2"] = d2.T @ h1
    g["b2"] = d2.sum(axis=0)
    d1 = (d2 @ p["W2"]) * (z1 > 0.0)
    g["W1"] = d1.T @ X
    g["b1"] = d1.sum(axis=0)
    grad = np.concatenate([g[name].ravel() for name, _ in shapes(n_in)])
    grad = grad + alpha / B * theta * mask
    return loss, grad


def adam_step(theta, m, v, t, g, lr, beta1, beta2, eps):
    t = t + 1
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    lrt = lr * np.sqrt(1.0 - beta2 ** t) / (1.0 - beta1 ** t)
    theta = theta - lrt * m / (np.sqrt(v) + eps)
    return theta, m, v, t


def train(theta0, X, y, order, lr=9e-4, beta1=0.95, beta2=0.90, eps=1e-9, alpha=1e-4, tol=1e-6,
          batch=200, max_epochs=200, n_iter_no_change=10, m0=None, v0=None, t0=0):
    """Minibatch Adam; order[e] is the row permutation of epoch e.

    Returns (theta, epoch_losses, epochs_run, m, v, t)."""
    theta = np.array(theta0, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n = X.shape[0]
    m = np.zeros_like(theta) if m0 is None else np.array(m0, dtype=np.float64)
    v = np.zeros_like(theta) if v0 is None else np.array(v0, dtype=np.float64)
    t = t0
    losses = []
    best = np.inf
    noimp = 0
    for e in range(max_epochs):
        acc = 0.0
        perm = np.asarray(order[e])
        for start in range(0, n, batch):
            rows = perm[start:start + batch]
            lb, g = loss_grad(theta, X[rows], y[rows], alpha)
            acc += lb * len(rows)
            theta, m, v, t = adam_step(theta, m, v, t, g, lr, beta1, beta2, eps)
        el = acc / n
        losses.append(el)
        if el > best - tol:
            noimp += 1
        else:
            noimp = 0
        if el < best:
            best = el
        if noimp > n_iter_no_change:
            break
    return theta, np.array(losses), len(losses), m, v, t


def standard_scaler(F):
    """Mean and (population) standard deviation per column; 0 -> 1."""
    F = np.asarray(F, dtype=np.float64)
    mean = F.mean(axis=0)
    std = F.std(axis=0)
    std = np.where(std == 0.0, 1.0, std)
    return mean, std


def r2(y, yhat):
    """Coefficient of determination, Eq. (R_square)."""
    y = np.asarray(y, dtype=np.float64)
    yhat = np.asarray(yhat, dtype=np.float64)
    return 1.0 - np.sum((y - yhat) ** 2) / np.sum((y - y.mean()) ** 2)


def decode(idx, radix):
    """Mixed-radix digits of idx, first digit fastest."""
    out = []
    for r in radix:
        out.append(idx % r)
        idx //= r
    return out


def features(params14, mean, std):
    """Standardised log2 of the 14 launch parameters, one row per vector."""
    P = np.asarray(params14, dtype=np.float64)
    return (np.log2(P) - mean) / std
