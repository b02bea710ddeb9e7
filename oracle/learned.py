"""Learned correction stage of the preconditioner (a project extension; the
paper has no learned component).  FP64 throughout; TEST INFRASTRUCTURE ONLY.

What is computed, in order (readings of this project, not the paper's):

* Grid mapping.  The DG coefficient vector on n^3 cells of degree k
  (cell-blocked, cell c = cx + n cy + n^2 cz, local node i + N j + N^2 l,
  N = k + 1) is a G^3 grid with G = n N: node (i, j, l) of cell
  (cx, cy, cz) sits at grid point (gx, gy, gz) = (N cx + i, N cy + j,
  N cz + l).  Grids are stored as arrays indexed [gz, gy, gx].
* Network.  Four 3x3x3 convolutions 1 -> C -> C -> C -> 1 (cross-correlation,
  zero padding of one point, bias), ReLU after the first three.  Weights are
  indexed w[c_out, c_in, dz, dy, dx] with offset index 0 meaning -1.  The
  network output is multiplied by a fixed power of two sigma that is chosen
  once from training data (so targets and outputs have similar size).
* Stage.  For a Krylov vector v: z = V(v) (the multigrid V-cycle); the
  residual rho = v - A z; s = 2^ceil(log2 max|rho|); the correction
  c = s * sigma * net(grid(rho / s)) (mapped back to cells); q = A c; the
  corrected z + alpha c with alpha = (rho . q) / (q . q), the factor that
  minimises ||v - A (z + alpha c)||_2 (alpha = 0 if q = 0).  If rho = 0 the
  correction is zero.  (The factor keeps a correction whose error is rich
  in high frequencies, which A amplifies, from raising the residual.)
* Fallback.  The solve switches to the plain V-cycle for all later
  iterations as soon as one iteration reduces the residual estimate by a
  factor worse than 0.9, or a corrected vector is not finite (that
  iteration then uses the plain V-cycle result).
* Training pairs.  Starting from x (an approximate solution of A x = b for a
  smooth right-hand side), each pair of a chain is r = A x, z = V(r),
  e = x - z, rho = r - A z (so A e = rho), scaled by s = 2^ceil(log2
  max|rho|): input rho / s, target e / s.  The next x of the chain is
  e / 2^ceil(log2 max|e|), the post-V-cycle error, which is what the later
  Krylov vectors of the solve contain.
* Loss.  Masked mean squared error sum(m (sigma y - t)^2) / sum(m), m >= 0.
* Optimizer.  Adam (Kingma and Ba 2015, Alg. 1), beta1 = 0.9,
  beta2 = 0.999, eps = 1e-8, bias-corrected moments.
* Crops.  Training may use cubes of side c cut from the G^3 pair grids; the
  loss mask then drops the points closer than the network's receptive
  radius (4) to a crop face that lies inside the full grid, where the crop's
  zero padding differs from the full grid's neighbours.
"""
import numpy as np

from . import fgmres as _fgmres

PARAM_NAMES = ("w1", "b1", "w2", "b2", "w3", "b3", "w4", "b4")
RECEPTIVE_RADIUS = 4


# ---------------------------------------------------------------------------
# Grid mapping
# ---------------------------------------------------------------------------

def cells_to_grid(u, n, k):
    N = k + 1
    G = n * N
    return (np.asarray(u).reshape(n, n, n, N, N, N)      # [cz, cy, cx, l, j, i]
            .transpose(0, 3, 1, 4, 2, 5).reshape(G, G, G))


def grid_to_cells(g, n, k):
    N = k + 1
    return (np.asarray(g).reshape(n, N, n, N, n, N)      # [cz, l, cy, j, cx, i]
            .transpose(0, 2, 4, 1, 3, 5).reshape(-1))


# ---------------------------------------------------------------------------
# Network
# ---------------------------------------------------------------------------

def param_shapes(C=32):
    return {"w1": (C, 1, 3, 3, 3), "b1": (C,), "w2": (C, C, 3, 3, 3), "b2": (C,),
            "w3": (C, C, 3, 3, 3), "b3": (C,), "w4": (1, C, 3, 3, 3), "b4": (1,)}


def flatten(params):
    """Parameters in the order w1 b1 w2 b2 w3 b3 w4 b4, each C-ordered."""
    return np.concatenate([np.asarray(params[k], dtype=np.float64).ravel() for k in PARAM_NAMES])


def unflatten(flat, C=32):
    out, o = {}, 0
    for name in PARAM_NAMES:
        shp = param_shapes(C)[name]
        m = int(np.prod(shp))
        out[name] = np.asarray(flat[o:o + m], dtype=np.float64).reshape(shp)
        o += m
    if o != len(flat):
        raise ValueError("parameter vector has the wrong length")
    return out


def conv3d(x, w, b):
    """y[co] = b[co] + sum_{ci, a, b, c} w[co, ci, a, b, c] xp[ci, z+a, y+b, x+c],
    xp = x padded with one zero on every face."""
    cin, G = x.shape[0], x.shape[1]
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (1, 1)))
    y = np.empty((w.shape[0], G, G, G))
    y[:] = np.asarray(b)[:, None, None, None]
    for a in range(3):
        for bb in range(3):
            for c in range(3):
                sl = xp[:, a:a + G, bb:bb + G, c:c + G].reshape(cin, -1)
                y += (w[:, :, a, bb, c] @ sl).reshape(y.shape)
    return y


def conv3d_backward(x, w, gy):
    """Gradients of sum(gy * conv3d(x, w, b)) with respect to x, w and b."""
    G = x.shape[1]
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (1, 1)))
    gxp = np.zeros_like(xp)
    gw = np.zeros_like(w)
    gy2 = gy.reshape(gy.shape[0], -1)
    for a in range(3):
        for bb in range(3):
            for c in range(3):
                sl = (slice(None), slice(a, a + G), slice(bb, bb + G), slice(c, c + G))
                gw[:, :, a, bb, c] = gy2 @ xp[sl].reshape(xp.shape[0], -1).T
                gxp[sl] += (w[:, :, a, bb, c].T @ gy2).reshape((w.shape[1],) + gy.shape[1:])
    return gxp[:, 1:-1, 1:-1, 1:-1], gw, gy.sum(axis=(1, 2, 3))


def forward(params, x):
    """Network output (before sigma) on one grid x [G, G, G] and the layer
    inputs a0..a3 (a1..a3 after ReLU)."""
    a0 = np.asarray(x, dtype=np.float64)[None]
    a1 = np.maximum(conv3d(a0, params["w1"], params["b1"]), 0.0)
    a2 = np.maximum(conv3d(a1, params["w2"], params["b2"]), 0.0)
    a3 = np.maximum(conv3d(a2, params["w3"], params["b3"]), 0.0)
    y = conv3d(a3, params["w4"], params["b4"])[0]
    return y, (a0, a1, a2, a3)


def masked_mse(y, t, mask, sigma):
    m = np.asarray(mask, dtype=np.float64)
    return float(np.sum(m * (sigma * y - t) ** 2) / np.sum(m))


def loss_and_grads(params, sigma, xs, ts, masks):
    """Masked MSE over a batch of grids (one mask per grid; the loss is the
    masked sum over the whole batch divided by the total mask weight) and its
    exact gradient with respect to every parameter."""
    total = float(sum(np.sum(m) for m in masks))
    loss = 0.0
    grads = {k: np.zeros_like(v) for k, v in params.items()}
    for x, t, m in zip(xs, ts, masks):
        y, acts = forward(params, x)
        d = sigma * y - t
        loss += float(np.sum(m * d * d)) / total
        gy = (2.0 * sigma / total) * m * d
        for name, g in _backprop(params, acts, gy).items():
            grads[name] += g
    return loss, grads


def _backprop(params, acts, gy):
    """Parameter gradients of one grid from the output gradient gy (chain
    rule through the four convolutions and the ReLUs)."""
    a0, a1, a2, a3 = acts
    g3, gw4, gb4 = conv3d_backward(a3, params["w4"], gy[None])
    g3 = g3 * (a3 > 0)
    g2, gw3, gb3 = conv3d_backward(a2, params["w3"], g3)
    g2 = g2 * (a2 > 0)
    g1, gw2, gb2 = conv3d_backward(a1, params["w2"], g2)
    g1 = g1 * (a1 > 0)
    _, gw1, gb1 = conv3d_backward(a0, params["w1"], g1)
    return {"w1": gw1, "b1": gb1, "w2": gw2, "b2": gb2, "w3": gw3, "b3": gb3, "w4": gw4,
            "b4": gb4}


def residual_loss_and_grads(params, sigma, A, rho_grids, n, k):
    """Residual-aware loss of the stage (a project reading: the stage should
    cancel the post-V-cycle residual, not match the error pointwise, since A
    amplifies the high-frequency part of any error in e).  For scaled
    residual grids rho_p (input) the correction c_p = sigma net(rho_p) is
    mapped to cells, q_p = A c_p, and the loss is what the stage itself
    leaves, with its own step length alpha_p = (rho_p . q_p) / (q_p . q_p)
    (0 when q_p = 0), the minimiser of ||rho_p - alpha q_p||:
        L = sum_p ||r_p||^2 / sum_p ||rho_p||^2,  r_p = rho_p - alpha_p q_p.
    Gradient: at the minimising alpha the derivative in alpha vanishes, so
    dL/dq_p = -2 alpha_p r_p / sum ||rho||^2 and, A being symmetric,
    dL/dy_p = -2 sigma alpha_p grid(A r_p) / sum_p ||rho_p||^2, propagated
    through the network as in loss_and_grads.  The loss does not depend on
    sigma (alpha absorbs any scale of the output)."""
    total = float(sum(np.sum(np.asarray(g) ** 2) for g in rho_grids))
    loss = 0.0
    grads = {key: np.zeros_like(v) for key, v in params.items()}
    for g in rho_grids:
        y, acts = forward(params, g)
        rho = grid_to_cells(g, n, k)
        q = A @ (sigma * grid_to_cells(y, n, k))
        qq = float(q @ q)
        alpha = float(rho @ q) / qq if qq > 0.0 else 0.0
        r = rho - alpha * q
        loss += float(r @ r) / total
        gy = (-2.0 * sigma * alpha / total) * cells_to_grid(A @ r, n, k)
        for name, gg in _backprop(params, acts, gy).items():
            grads[name] += gg
    return loss, grads


class Adam:
    def __init__(self, n, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.beta1, self.beta2, self.eps = lr, beta1, beta2, eps

    def step(self, theta, g):
        self.t += 1
        self.m = self.beta1 * self.m + (1.0 - self.beta1) * g
        self.v = self.beta2 * self.v + (1.0 - self.beta2) * g * g
        mhat = self.m / (1.0 - self.beta1 ** self.t)
        vhat = self.v / (1.0 - self.beta2 ** self.t)
        return theta - self.lr * mhat / (np.sqrt(vhat) + self.eps)


# ---------------------------------------------------------------------------
# Crops
# ---------------------------------------------------------------------------

def crop(grid, off, c):
    z, y, x = off
    return grid[z:z + c, y:y + c, x:x + c]


def crop_mask(G, off, c, radius=RECEPTIVE_RADIUS):
    """1 where a crop point's network output equals the full grid's: at
    least `radius` points away from every crop face inside the full grid."""
    m1 = []
    for o in off:
        w = np.ones(c)
        if o > 0:
            w[:radius] = 0.0
        if o + c < G:
            w[c - radius:] = 0.0
        m1.append(w)
    return m1[0][:, None, None] * m1[1][None, :, None] * m1[2][None, None, :]


# ---------------------------------------------------------------------------
# Solver-generated pairs and the learned preconditioner
# ---------------------------------------------------------------------------

def pow2_ceil(v):
    """2^ceil(log2 v) for v > 0."""
    m, e = np.frexp(v)          # v = m 2^e, m in [0.5, 1)
    return float(np.ldexp(1.0, int(e) - (1 if m == 0.5 else 0)))


def make_pairs(A, precondition, x, count, n, k):
    """A chain of `count` training pairs (rho / s, e / s, s) as grids."""
    out = []
    x = np.array(x, dtype=np.float64)
    for _ in range(count):
        r = A @ x
        z = precondition(r)
        e = x - z
        rho = r - A @ z
        s = pow2_ceil(np.abs(rho).max())
        out.append((cells_to_grid(rho / s, n, k), cells_to_grid(e / s, n, k), s))
        x = e / pow2_ceil(np.abs(e).max())
    return out


def learned_precondition(A, precondition, net, n, k):
    """z -> the stage of the module docstring; `net(grid)` returns
    sigma * network(grid)."""
    def apply(v):
        z = precondition(v)
        rho = v - A @ z
        mx = np.abs(rho).max()
        if mx == 0.0:
            return z
        s = pow2_ceil(mx)
        c = s * grid_to_cells(net(cells_to_grid(rho / s, n, k)), n, k)
        q = A @ c
        qq = float(q @ q)
        alpha = float(rho @ q) / qq if qq > 0.0 else 0.0
        return z + alpha * c
    return apply


def solve(A, b, precondition, net, n, k, rtol=1e-10, restart=30, max_iters=300,
          stagnation=0.9):
    """FGMRES with the learned stage and its fallback to the plain V-cycle.
    Returns (x, info) with info['fell_back'] added."""
    learned = learned_precondition(A, precondition, net, n, k)
    state = {"fell_back": False}

    def precond(v):
        if state["fell_back"]:
            return precondition(v)
        z = learned(v)
        if not np.all(np.isfinite(z)):
            state["fell_back"] = True
            return precondition(v)
        return z

    def watch(history):
        if len(history) >= 2 and not state["fell_back"]:
            prev, cur = history[-2], history[-1]
            if not np.isfinite(cur) or cur > stagnation * prev:
                state["fell_back"] = True

    x, info = _fgmres.fgmres(lambda v: A @ v, b, precond, rtol=rtol, restart=restart,
                             max_iters=max_iters, on_estimate=watch)
    info["fell_back"] = state["fell_back"]
    return x, info


def network_fn(params, sigma):
    return lambda g: sigma * forward(params, g)[0]
