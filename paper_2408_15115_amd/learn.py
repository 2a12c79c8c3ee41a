"""Training loop of the learned warm start (orchestration only).

Samples come from the solver's own plain runs (lbm_ibm_samples); the network
is trained by the library's forward/backward kernels and Adam.  Features and
targets are standardized on the host for training, and the standardization
is folded into the first and last layers afterwards, so the device network
maps raw features to raw targets.
"""
from __future__ import annotations

import numpy as np

from . import turret as T

_SHAPES = [(T.MLP_IN, 64), (64, 64), (64, 3)]


def _split(theta):
    out, k = [], 0
    for i, o in _SHAPES:
        W = theta[k:k + o * i].reshape(o, i)
        k += o * i
        out.append([W, theta[k:k + o]])
        k += o
    return out


def collect(solver, steps, skip=10):
    """Run `steps` coupled steps; return host arrays (features, targets) of
    every step after the first `skip`."""
    X, Y = [], []
    for n in range(steps):
        solver.run(1)
        if n >= skip:
            f, t = solver.ibm_samples()
            X.append(f.cpu().numpy())
            Y.append(t.cpu().numpy())
    return np.concatenate(X), np.concatenate(Y)


def fit(net, X, Y, iters=2500, batch=8192, lr=1e-3, lr_final=3e-4, seed=0):
    """Train `net` on (X, Y); returns the last mini-batch loss (standardized
    units).  The network ends up mapping raw X to raw Y."""
    import torch
    # the std floor keeps the folded first-layer weights inside FP16 range
    mx, sx = X.mean(0), np.maximum(X.std(0), 1e-4)
    my, sy = Y.mean(0), Y.std(0) + 1e-9
    Xd = torch.tensor(((X - mx) / sx).astype(np.float32), device="cuda")
    Yd = torch.tensor(((Y - my) / sy).astype(np.float32), device="cuda")
    gen = torch.Generator(device="cuda").manual_seed(seed)
    loss = torch.zeros(1, device="cuda")
    batch = min(batch, X.shape[0], net.max_batch)
    for it in range(iters):
        idx = torch.randint(0, Xd.shape[0], (batch,), device="cuda", generator=gen)
        net.train_step(Xd[idx].contiguous(), Yd[idx].contiguous(), lr=lr if it < 0.7 * iters else lr_final,
                       loss=loss)
    theta = net.params().astype(np.float64)
    (W1, b1), mid, (W3, b3) = _split(theta)
    # the device rounds weights to FP16: fold the input mean with the
    # rounded first-layer weights so that only (x - mean) sees their rounding
    W1n = (W1 / sx[None, :]).astype(np.float16).astype(np.float64)
    b1n = b1 - W1n @ mx
    W3n = W3 * sy[:, None]
    b3n = b3 * sy + my
    folded = np.concatenate([W1n.ravel(), b1n, mid[0].ravel(), mid[1], W3n.ravel(), b3n]).astype(np.float32)
    net.set_params(folded)
    return float(loss.item())
