"""Learned preconditioner: 3D convolutions, the U-Net, its loss and gradients, Adam, and
flexible CG (oracle, float64, CPU).

The paper has no learned component; its Sec. "Path to Geometric Multigrid Integration"
names better preconditioning as the way past Jacobi-PCG's iteration counts.  This module
is the plain definition of the network the library trains (3 levels, 16 base
channels, inputs residual xyz + nodal density on the node grid, output a correction)
and of flexible CG (Notay's FCG with truncation 1), written as direct sums so that the
GPU kernels can be checked against them.  Parity of the network's *value as a
preconditioner* is unpinned (it is learned); its forward and backward passes are pinned
by a library convolution and by finite differences in tests/test_oracle_nn.py.

Tensors are (C, D, H, W) = (channels, z, y, x) on the node grid.
"""
from __future__ import annotations

import numpy as np

LEAK = 0.01


# -------------------------------------------------------------------- convolutions
def out_size(n: int, stride: int) -> int:
    """Output length of a 3-tap convolution with zero padding 1 and the given stride."""
    return (n - 1) // stride + 1


def conv3d(x: np.ndarray, w: np.ndarray, stride: int = 1) -> np.ndarray:
    """y[o, d, h, w] = sum_{i, a, b, c} W[o, i, a, b, c] x[i, s d + a - 1, s h + b - 1, s w + c - 1]
    with zero padding (taps outside the grid contribute nothing)."""
    C, D, H, W_ = x.shape
    O = w.shape[0]
    kz, ky, kx = w.shape[2:]
    pz, py, px = kz // 2, ky // 2, kx // 2
    Do, Ho, Wo = out_size(D, stride), out_size(H, stride), out_size(W_, stride)
    xp = np.zeros((C, D + 2 * pz, H + 2 * py, W_ + 2 * px))
    xp[:, pz:pz + D, py:py + H, px:px + W_] = x
    y = np.zeros((O, Do, Ho, Wo))
    for a in range(kz):
        for b in range(ky):
            for c in range(kx):
                sl = xp[:, a:a + stride * (Do - 1) + 1:stride,
                        b:b + stride * (Ho - 1) + 1:stride,
                        c:c + stride * (Wo - 1) + 1:stride]
                y += np.einsum("oi,idhw->odhw", w[:, :, a, b, c], sl)
    return y


def conv3d_bwd_data(dy: np.ndarray, w: np.ndarray, in_shape, stride: int = 1) -> np.ndarray:
    """Adjoint of conv3d with respect to x: scatter every output gradient back to the
    taps that produced it."""
    C, D, H, W_ = in_shape
    kz, ky, kx = w.shape[2:]
    pz, py, px = kz // 2, ky // 2, kx // 2
    Do, Ho, Wo = dy.shape[1:]
    dxp = np.zeros((C, D + 2 * pz, H + 2 * py, W_ + 2 * px))
    for a in range(kz):
        for b in range(ky):
            for c in range(kx):
                dxp[:, a:a + stride * (Do - 1) + 1:stride,
                    b:b + stride * (Ho - 1) + 1:stride,
                    c:c + stride * (Wo - 1) + 1:stride] += np.einsum(
                        "oi,odhw->idhw", w[:, :, a, b, c], dy)
    return dxp[:, pz:pz + D, py:py + H, px:px + W_]


def conv3d_bwd_weight(x: np.ndarray, dy: np.ndarray, ksize: int, stride: int = 1) -> np.ndarray:
    """dW[o, i, a, b, c] = sum over outputs of dy[o, .] x[i, tap (a, b, c) of that output]."""
    C, D, H, W_ = x.shape
    p = ksize // 2
    Do, Ho, Wo = dy.shape[1:]
    xp = np.zeros((C, D + 2 * p, H + 2 * p, W_ + 2 * p))
    xp[:, p:p + D, p:p + H, p:p + W_] = x
    dw = np.zeros((dy.shape[0], C, ksize, ksize, ksize))
    for a in range(ksize):
        for b in range(ksize):
            for c in range(ksize):
                sl = xp[:, a:a + stride * (Do - 1) + 1:stride,
                        b:b + stride * (Ho - 1) + 1:stride,
                        c:c + stride * (Wo - 1) + 1:stride]
                dw[:, :, a, b, c] = np.einsum("odhw,idhw->oi", dy, sl)
    return dw


def leaky(x):
    return np.where(x > 0, x, LEAK * x)


def leaky_grad(x, g):
    return np.where(x > 0, g, LEAK * g)


def upsample(x: np.ndarray, shape) -> np.ndarray:
    """Nearest-neighbour up-sampling by 2 cropped to `shape`: out[., d, h, w] =
    x[., d // 2, h // 2, w // 2]."""
    D, H, W_ = shape
    return x[:, np.arange(D) // 2][:, :, np.arange(H) // 2][:, :, :, np.arange(W_) // 2]


def upsample_adjoint(g: np.ndarray, coarse_shape) -> np.ndarray:
    out = np.zeros((g.shape[0],) + tuple(coarse_shape))
    D, H, W_ = g.shape[1:]
    dz, dy, dx = np.arange(D) // 2, np.arange(H) // 2, np.arange(W_) // 2
    for i in range(D):
        for j in range(H):
            np.add.at(out[:, dz[i], dy[j], :], (slice(None), dx), g[:, i, j, :])
    return out


# -------------------------------------------------------------------------- U-Net
# Layers in execution order: (name, c_in, c_out, kernel, stride).  Level 0 has `base`
# channels, level 1 2*base, level 2 4*base; skips are concatenated [up, skip].
def unet_layers(base: int = 16, cin: int = 4, cout: int = 3):
    b1, b2, b3 = base, 2 * base, 4 * base
    return [
        ("e0a", cin, b1, 3, 1), ("e0b", b1, b1, 3, 1),
        ("d1", b1, b2, 3, 2), ("e1", b2, b2, 3, 1),
        ("d2", b2, b3, 3, 2), ("m2a", b3, b3, 3, 1), ("m2b", b3, b3, 3, 1),
        ("u1a", b3 + b2, b2, 3, 1), ("u1b", b2, b2, 3, 1),
        ("u0a", b2 + b1, b1, 3, 1), ("u0b", b1, b1, 3, 1),
        ("head", b1, cout, 1, 1),
    ]


def unet_init(base=16, cin=4, cout=3, seed=0):
    """He-normal initial weights (fan-in = c_in k^3), no biases."""
    rng = np.random.default_rng(seed)
    params = {}
    for name, ci, co, k, _ in unet_layers(base, cin, cout):
        std = np.sqrt(2.0 / (ci * k ** 3))
        params[name] = rng.standard_normal((co, ci, k, k, k)) * std
    return params


def unet_forward(params, x, base=16):
    """Forward pass; returns (output, cache of pre-activations and layer inputs)."""
    L = {n: (ci, co, k, s) for n, ci, co, k, s in unet_layers(base, x.shape[0],
                                                               params["head"].shape[0])}
    cache = {}

    def layer(name, inp, act=True):
        z = conv3d(inp, params[name], L[name][3])
        cache[name] = (inp, z)
        return leaky(z) if act else z

    a = layer("e0a", x)
    s0 = layer("e0b", a)
    a = layer("d1", s0)
    s1 = layer("e1", a)
    a = layer("d2", s1)
    a = layer("m2a", a)
    a = layer("m2b", a)
    a = np.concatenate([upsample(a, s1.shape[1:]), s1], axis=0)
    a = layer("u1a", a)
    a = layer("u1b", a)
    a = np.concatenate([upsample(a, s0.shape[1:]), s0], axis=0)
    a = layer("u0a", a)
    a = layer("u0b", a)
    out = layer("head", a, act=False)
    cache["shapes"] = (s0.shape, s1.shape, cache["m2b"][1].shape)
    return out, cache


def unet_backward(params, cache, dout, base=16):
    """Gradients of a scalar loss with respect to every weight, given dLoss/dout."""
    L = {n: (ci, co, k, s) for n, ci, co, k, s in unet_layers(base, cache["e0a"][0].shape[0],
                                                               params["head"].shape[0])}
    grads = {}

    def back(name, g, act=True):
        inp, z = cache[name]
        gz = leaky_grad(z, g) if act else g
        grads[name] = conv3d_bwd_weight(inp, gz, L[name][2], L[name][3])
        return conv3d_bwd_data(gz, params[name], inp.shape, L[name][3])

    s0_shape, s1_shape, m2_shape = cache["shapes"]
    b1, b2 = base, 2 * base
    g = back("head", dout, act=False)
    g = back("u0b", g)
    g = back("u0a", g)                       # gradient wrt [up(u1b), s0]
    g_up0, g_s0 = g[:b2], g[b2:]
    g = upsample_adjoint(g_up0, s1_shape[1:])
    g = back("u1b", g)
    g = back("u1a", g)                       # gradient wrt [up(m2b), s1]
    g_up1, g_s1 = g[:4 * base], g[4 * base:]
    g = upsample_adjoint(g_up1, m2_shape[1:])
    g = back("m2b", g)
    g = back("m2a", g)
    g = back("d2", g)
    g = g + g_s1
    g = back("e1", g)
    g = back("d1", g)
    g = g + g_s0
    g = back("e0b", g)
    back("e0a", g)
    return grads


def rel_mse_loss(out, target, mask):
    """sum(mask (out - target)^2) / sum(mask target^2) and its gradient wrt out."""
    d = (out - target) * mask
    den = np.sum((target * mask) ** 2)
    return float(np.sum(d * d) / den), 2.0 * d * mask / den


def energy_loss(n, r, e, apply_K, free):
    """Relative energy-norm error of the best multiple of the correction n:
    with a = <n, r>, q = <n, K n>, c = <e, r> (e = K^-1 r, so c = ||e||_K^2),
    L = min_s ||s n - e||_K^2 / ||e||_K^2 = 1 - a^2 / (q c),
    and dL/dn = -(2 a / (q c)) (r - (a / q) K n), on free DOFs (n is masked first)."""
    n = n * free
    Kn = apply_K(n)
    a, q, c = float(n @ r), float(n @ Kn), float(e @ r)
    if not (q > 0 and c > 0):
        return 1.0, np.zeros_like(n)
    L = 1.0 - a * a / (q * c)
    g = -(2.0 * a / (q * c)) * (r - (a / q) * Kn) * free
    return L, g


def adam_step(params, grads, state, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected moments) of every parameter, in place."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in params:
        m = state.setdefault("m_" + k, np.zeros_like(params[k]))
        v = state.setdefault("v_" + k, np.zeros_like(params[k]))
        m *= b1
        m += (1 - b1) * grads[k]
        v *= b2
        v += (1 - b2) * grads[k] ** 2
        mhat = m / (1 - b1 ** t)
        vhat = v / (1 - b2 ** t)
        params[k] -= lr * mhat / (np.sqrt(vhat) + eps)
    return params


# ------------------------------------------------------------------ flexible CG
def fcg(apply_A, precond, b, x0=None, tol=1e-8, maxit=10000, window=1, d=None, stall=0,
        info=None):
    """Flexible CG truncated to the `window` latest directions (FCG(m)): z_k = M_k(r_k),
    p_k = z_k - sum_j (<z_k, q_j> / <p_j, q_j>) p_j over the window, q_k = A p_k,
    alpha_k = <r_k, z_k> / <p_k, q_k>.  With a fixed SPD preconditioner this reproduces
    PCG in exact arithmetic for every window.  Stops on ||r|| <= tol ||b||.

    Guards of the learned preconditioner (plain Jacobi-PCG is its fallback):
      * with the Jacobi diagonal `d`: a z that is not a descent direction (<r, z> <= 0),
        is not finite, or gives a non-finite orthogonalisation coefficient is replaced by
        the Jacobi step z = r / d for that iteration (counted in info["fallbacks"]);
      * with stall > 0: once ||r|| has made no new minimum for `stall` consecutive
        iterations, flexible CG stops and plain Jacobi-PCG (solvers.pcg_jacobi, needs d)
        continues from the current iterate with the same tolerance on ||b|| and the
        iterations left (info["restarted"] = True, info["fcg_iterations"] = iterations
        flexible CG took).
    Returns (x, iters, history); iters and history include the Jacobi-PCG part."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    bn = np.linalg.norm(b)
    r = b - apply_A(x)
    hist = [np.linalg.norm(r) / bn]
    P, Q = [], []
    it = 0
    fallbacks = 0
    best, k_best = hist[0], 0
    restarted = False
    while hist[-1] > tol and it < maxit:
        z = precond(r)
        with np.errstate(all="ignore"):
            rz = float(r @ z)
            coef = [float(z @ qj) / float(pj @ qj) for pj, qj in zip(P, Q)]
        ok = np.isfinite(rz) and rz > 0.0 and all(np.isfinite(c) for c in coef)
        if not ok and d is not None:
            z = r / d
            fallbacks += 1
            coef = [float(z @ qj) / float(pj @ qj) for pj, qj in zip(P, Q)]
        p = z.copy()
        for c, pj in zip(coef, P):
            p -= c * pj
        q = apply_A(p)
        alpha = (r @ z) / (p @ q)
        x = x + alpha * p
        r = r - alpha * q
        P.append(p)
        Q.append(q)
        if len(P) > window:
            P.pop(0)
            Q.pop(0)
        it += 1
        hist.append(np.linalg.norm(r) / bn)
        if stall > 0 and hist[-1] > tol and it < maxit:
            if hist[-1] < best:
                best, k_best = hist[-1], it
            elif it - k_best >= stall:
                restarted = True
                break
    fcg_its = it
    if restarted and it < maxit:
        from oracle.solvers import pcg_jacobi
        x, it2, h2 = pcg_jacobi(apply_A, d, b, x, tol, maxit - it)
        it += it2
        hist.extend(h2[1:])
    if info is not None:
        info.update(fallbacks=fallbacks, restarted=restarted, fcg_iterations=fcg_its)
    return x, it, hist


def node_density(xphys: np.ndarray, nx: int, ny: int, nz: int) -> np.ndarray:
    """Mean density of the (up to eight) elements around each node, shape (nz+1, ny+1, nx+1)."""
    e = xphys.reshape(nz, ny, nx)
    s = np.zeros((nz + 1, ny + 1, nx + 1))
    c = np.zeros_like(s)
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                s[dz:dz + nz, dy:dy + ny, dx:dx + nx] += e
                c[dz:dz + nz, dy:dy + ny, dx:dx + nx] += 1
    return s / c


def nn_precondition(params, r: np.ndarray, rho_node: np.ndarray, fixed_mask: np.ndarray,
                    base=16) -> np.ndarray:
    """z = (||r|| / sqrt(n)) N([r sqrt(n) / ||r||, rho_node]) on the node grid (n = r.size:
    the residual channels enter at unit RMS, the scale of the density channel), zero on
    fixed DOFs.  Homogeneous of degree one in r."""
    D, H, W_ = rho_node.shape
    rn = np.linalg.norm(r)
    if rn == 0:
        return np.zeros_like(r)
    g = np.sqrt(r.size) / rn
    rr = (r * g).reshape(D, H, W_, 3).transpose(3, 0, 1, 2)
    inp = np.concatenate([rr, rho_node[None]], axis=0)
    out, _ = unet_forward(params, inp, base)
    z = out.transpose(1, 2, 3, 0).reshape(-1) / g
    z[fixed_mask] = 0.0
    return z


def two_stage(r: np.ndarray, n: np.ndarray, apply_K, d: np.ndarray) -> np.ndarray:
    """Correction n followed by a Jacobi step on the remaining residual:
    s = <r, n> / <n, K n> (the scale minimising the energy norm of the error after the
    correction; 0 unless both are positive), z = s n + D^-1 (r - s K n)."""
    Kn = apply_K(n)
    rn, nkn = float(r @ n), float(n @ Kn)
    s = rn / nkn if (rn > 0 and nkn > 0) else 0.0
    return s * n + (r - s * Kn) / d


def nn_two_stage_precondition(params, r, rho_node, fixed_mask, apply_K, d, base=16):
    """The learned preconditioner of the flexible CG: two_stage with n the network output."""
    n = nn_precondition(params, r, rho_node, fixed_mask, base)
    return two_stage(r, n, apply_K, d)

