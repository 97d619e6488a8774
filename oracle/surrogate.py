"""Reference forward pass, loss gradient and optimizer step of the stiffness surrogate (CPU, FP64).

TEST INFRASTRUCTURE ONLY (see the package header).

The surrogate maps a two-phase voxel cell and the phase moduli to the 21
independent components of the homogenized 6x6 stiffness (the quantity of
section 3.3, computed by the solver as training data).  The network is a plain
definition, written for checking by eye:

    a0 = phase indicator, channels-last [B, n, n, n, 1]
    a_l = gelu( conv_l(a_{l-1}) + b_l ),  l = 1..4
          conv_l: 3x3x3 kernel, stride 2, periodic wrap (the cell is periodic):
          out[b, o, co] = sum_{t in {0,1,2}^3} sum_ci W_l[co, t, ci] a[b, (2 o + t - 1) mod n, ci]
    g   = mean of a_4 over its voxels                              [B, 256]
    h   = gelu( [g, feat] W_5^T + b_5 )                            [B, 256]
    y   = h W_6^T + b_6                                            [B, 21]

with gelu(x) = x Phi(x) (the exact, erf-based form).  Loss: mean squared error
over the batch and the 21 outputs.  Gradients come from torch.autograd on this
forward definition in float64 (a library primitive differentiating exactly the
expression above); the tests pin the forward against brute-force loops and
closed forms, and the gradients against central finite differences.
Optimizer: Adam (Kingma & Ba 2015) with bias correction.
"""

import math

import numpy as np
import torch

CHANNELS = (1, 32, 64, 128, 256)
HIDDEN = 256
N_OUT = 21
N_FEAT = 1


def param_shapes(channels=CHANNELS, hidden=HIDDEN, n_feat=N_FEAT, n_out=N_OUT):
    """Ordered (name, shape) list of the flat parameter vector."""
    shapes = []
    for l in range(1, len(channels)):
        shapes.append(("W%d" % l, (channels[l], 27, channels[l - 1])))
        shapes.append(("b%d" % l, (channels[l],)))
    shapes.append(("W5", (hidden, channels[-1] + n_feat)))
    shapes.append(("b5", (hidden,)))
    shapes.append(("W6", (n_out, hidden)))
    shapes.append(("b6", (n_out,)))
    return shapes


def n_params(**kw):
    return sum(int(np.prod(s)) for _, s in param_shapes(**kw))


def unflatten(theta, **kw):
    out, k = {}, 0
    for name, s in param_shapes(**kw):
        m = int(np.prod(s))
        out[name] = theta[k:k + m].reshape(s)
        k += m
    return out


def gelu(x):
    return 0.5 * x * (1.0 + torch.erf(x / math.sqrt(2.0)))


def offsets():
    """The 27 kernel taps t = (tz, ty, tx), tz slowest."""
    return [(tz, ty, tx) for tz in range(3) for ty in range(3) for tx in range(3)]


def conv_s2(a, W, b):
    """Stride-2, 3x3x3, periodic convolution; a [B, n, n, n, Ci] -> [B, n/2, n/2, n/2, Co]."""
    n = a.shape[1]
    m = n // 2
    idx = [torch.tensor([(2 * o + t - 1) % n for o in range(m)]) for t in range(3)]
    out = b.reshape(1, 1, 1, 1, -1).expand(a.shape[0], m, m, m, W.shape[0]).clone()
    for k, (tz, ty, tx) in enumerate(offsets()):
        patch = a.index_select(1, idx[tz]).index_select(2, idx[ty]).index_select(3, idx[tx])
        out = out + torch.einsum("bzyxc,oc->bzyxo", patch, W[:, k, :])
    return out


def forward(theta, phase, feat, **kw):
    """theta: flat float64 tensor; phase [B, n, n, n] (0/1); feat [B, n_feat].  Returns y [B, n_out]."""
    P = unflatten(theta, **kw)
    a = phase.to(torch.float64).unsqueeze(-1)
    for l in range(1, 5):
        a = gelu(conv_s2(a, P["W%d" % l], P["b%d" % l]))
    g = a.mean(dim=(1, 2, 3))
    h = gelu(torch.cat([g, feat.to(torch.float64)], dim=1) @ P["W5"].T + P["b5"])
    return h @ P["W6"].T + P["b6"]


def loss(theta, phase, feat, target, **kw):
    y = forward(theta, phase, feat, **kw)
    return ((y - target) ** 2).mean()


def loss_and_grad(theta, phase, feat, target, **kw):
    """Mean squared error and its gradient with respect to the flat parameters (float64)."""
    th = torch.as_tensor(np.asarray(theta, dtype=np.float64)).clone().requires_grad_(True)
    L = loss(th, torch.as_tensor(np.asarray(phase)), torch.as_tensor(np.asarray(feat, dtype=np.float64)),
             torch.as_tensor(np.asarray(target, dtype=np.float64)), **kw)
    L.backward()
    return float(L.detach()), th.grad.numpy().copy()


def predict(theta, phase, feat, **kw):
    with torch.no_grad():
        y = forward(torch.as_tensor(np.asarray(theta, dtype=np.float64)), torch.as_tensor(np.asarray(phase)),
                    torch.as_tensor(np.asarray(feat, dtype=np.float64)), **kw)
    return y.numpy()


def adam_step(theta, m, v, grad, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


# ---------------------------------------------------------------------------
# targets: the 21 independent stiffness components
# ---------------------------------------------------------------------------
def upper_indices(n=6):
    return [(i, j) for i in range(n) for j in range(i, n)]


def stiffness_to_vector(C):
    """Upper triangle (row-major) of a symmetric 6x6 matrix (or a batch of them)."""
    C = np.asarray(C)
    return np.stack([C[..., i, j] for i, j in upper_indices()], axis=-1)


def vector_to_stiffness(v):
    v = np.asarray(v)
    C = np.zeros(v.shape[:-1] + (6, 6))
    for k, (i, j) in enumerate(upper_indices()):
        C[..., i, j] = v[..., k]
        C[..., j, i] = v[..., k]
    return C
