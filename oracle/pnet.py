"""Plain FP64 reference of the learned prolongation (test infrastructure only).

TEST INFRASTRUCTURE ONLY: used by the test-suite to check the HIP network
kernels; the product path never imports it.

The transfer operator of MGMC may be any full-rank P with Galerkin coarse
operators (the invariance theorem of Sec. 4.2 is proved for general
prolongations, and Sec. 3.1 notes the intergrid operators are not unique),
so P only affects efficiency.  Here P on the finest transfer comes from a
small convolutional network of the local coefficient, trained to reduce the
two-grid error.  The two-grid error propagator of the convergence analysis
(Sec. 4.3: X = S_post T S_pre with the coarse correction T = I - P A_c^{-1}
P^T A, eq. def-Tell, and an exact coarse solve) gives the loss

    L(P) = mean_e || S_b T S_f e ||_A^2 / || e ||_A^2,   A_c = P^T A P,

with S_f, S_b one noise-free forward / backward red-black Gauss-Seidel sweep
(the smoothers of the sampler's finest level).  With e_s = S_f e,
x = A_c^{-1} P^T A e_s, r = e_s - P x, W = S_b^T A S_b and y = A_c^{-1} P^T W r,

    dL/dP = -2 mean_e [ (W r - A P y) x^T + (A r) y^T ] / || e ||_A^2.

(Without the smoothers, L reduces to the fraction of e's energy the coarse
space misses; minimising that alone was found to slow the V-cycle down.)

Network (all arrays on the coarse grid, nc x nc, zero padding):
  input  24 channels: log a on the 12 x-faces and 12 y-faces around the
         3 x 3 fine block centred at fine node 2J;
  conv 3x3 24 -> 16, ReLU; conv 3x3 16 -> 16, ReLU; conv 3x3 16 -> 9;
  rho = softplus(out); the weight of coarse node J at fine node 2J + delta is
  rho_J(delta) / Z(2J + delta), Z summing rho over the coarse nodes covering
  that fine node (boundary ghosts count as 1), and 1 at delta = 0.  Equal rho
  reproduce multilinear interpolation exactly.
"""
import numpy as np

NIN, NHID, NOUT = 24, 16, 9
SHAPES = [(NHID, NIN, 9), (NHID,), (NHID, NHID, 9), (NHID,), (NOUT, NHID, 9), (NOUT,)]


def nparams():
    return int(sum(np.prod(s) for s in SHAPES))


def unpack(theta):
    out, at = [], 0
    for s in SHAPES:
        k = int(np.prod(s))
        out.append(np.asarray(theta[at:at + k], dtype=np.float64).reshape(s))
        at += k
    return out


def face_views(faces, n):
    per = (n + 1) * n
    ax = np.asarray(faces[:per], dtype=np.float64).reshape(n, n + 1)   # [y-1][face x]
    ay = np.asarray(faces[per:2 * per], dtype=np.float64).reshape(n + 1, n)  # [face y][x-1]
    return ax, ay


def features(faces, n):
    """[24][nc][nc]: log a on the faces around the fine 3x3 block of each coarse node."""
    nc = (n - 1) // 2
    ax, ay = face_views(faces, n)
    X = np.zeros((NIN, nc, nc))
    for Jy in range(1, nc + 1):
        for Jx in range(1, nc + 1):
            ch = 0
            for r in range(3):          # fine rows 2Jy-1 .. 2Jy+1
                for fi in range(4):     # x-faces 2Jx-2 .. 2Jx+1
                    X[ch, Jy - 1, Jx - 1] = np.log(ax[2 * Jy - 1 + r - 1, 2 * Jx - 2 + fi])
                    ch += 1
            for fr in range(4):         # y-faces 2Jy-2 .. 2Jy+1
                for cx in range(3):     # fine columns 2Jx-1 .. 2Jx+1
                    X[ch, Jy - 1, Jx - 1] = np.log(ay[2 * Jy - 2 + fr, 2 * Jx - 1 + cx - 1])
                    ch += 1
    return X


def conv3x3(X, W, b):
    cout, cin, _ = W.shape
    _, H, Wd = X.shape
    Xp = np.zeros((cin, H + 2, Wd + 2))
    Xp[:, 1:-1, 1:-1] = X
    out = np.zeros((cout, H, Wd)) + b[:, None, None]
    for t in range(9):
        dx, dy = t % 3 - 1, t // 3 - 1
        patch = Xp[:, 1 + dy:1 + dy + H, 1 + dx:1 + dx + Wd]
        out += np.einsum("oc,chw->ohw", W[:, :, t], patch)
    return out


def conv3x3_backward(X, W, dout):
    """Gradients of out = conv3x3(X, W, b) w.r.t. X, W and b."""
    cout, cin, _ = W.shape
    _, H, Wd = X.shape
    Xp = np.zeros((cin, H + 2, Wd + 2))
    Xp[:, 1:-1, 1:-1] = X
    dW = np.zeros_like(W)
    dXp = np.zeros_like(Xp)
    for t in range(9):
        dx, dy = t % 3 - 1, t // 3 - 1
        patch = Xp[:, 1 + dy:1 + dy + H, 1 + dx:1 + dx + Wd]
        dW[:, :, t] = np.einsum("ohw,chw->oc", dout, patch)
        dXp[:, 1 + dy:1 + dy + H, 1 + dx:1 + dx + Wd] += np.einsum("oc,ohw->chw", W[:, :, t], dout)
    return dXp[:, 1:-1, 1:-1], dW, dout.sum(axis=(1, 2))


def softplus(x):
    return np.log1p(np.exp(-np.abs(x))) + np.maximum(x, 0.0)


def forward(theta, X):
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    z1 = conv3x3(X, W1, b1)
    a1 = np.maximum(z1, 0.0)
    z2 = conv3x3(a1, W2, b2)
    a2 = np.maximum(z2, 0.0)
    o = conv3x3(a2, W3, b3)
    return o, (X, z1, a1, z2, a2)


def covering(i, nc):
    """Coarse nodes J (1-based, may be ghosts 0 or nc+1) with fine i = 2J + d."""
    if i % 2 == 0:
        return [(i // 2, 0)]
    return [((i - 1) // 2, 1), ((i + 1) // 2, -1)]


def normalize(o, nc):
    """rho = softplus(o); w[J][t] = rho_J(t) / Z(2J + delta_t), w[J][centre] = 1.
    Returns w with shape [nc][nc][9] (t = (dx+1) + 3 (dy+1))."""
    rho = softplus(o)  # [9][nc][nc]

    def rho_at(Jy, Jx, dx, dy):
        if Jx < 1 or Jx > nc or Jy < 1 or Jy > nc:
            return 1.0
        return rho[(dx + 1) + 3 * (dy + 1), Jy - 1, Jx - 1]

    w = np.zeros((nc, nc, 9))
    for Jy in range(1, nc + 1):
        for Jx in range(1, nc + 1):
            for t in range(9):
                dx, dy = t % 3 - 1, t // 3 - 1
                if dx == 0 and dy == 0:
                    w[Jy - 1, Jx - 1, t] = 1.0
                    continue
                ix, iy = 2 * Jx + dx, 2 * Jy + dy
                Z = sum(rho_at(Ky, Kx, ex, ey) for Ky, ey in covering(iy, nc) for Kx, ex in covering(ix, nc))
                w[Jy - 1, Jx - 1, t] = rho_at(Jy, Jx, dx, dy) / Z
    return w


def prolongation_weights(theta, faces, n):
    """Learned weights in the layout of the library's prolong_w: [nc*nc][9]."""
    nc = (n - 1) // 2
    o, _ = forward(theta, features(faces, n))
    return normalize(o, nc).reshape(nc * nc, 9)


def fine_operator_dense(faces, n, kappa2, ix0, iy0, width, scale=None):
    """The finite-difference operator on the fine window [ix0, ix0+width) x
    [iy0, iy0+width) with zero Dirichlet data outside the window."""
    h = 1.0 / (n + 1)
    s = h * h if scale is None else scale
    ax, ay = face_views(faces, n)
    m = width * width
    A = np.zeros((m, m))
    for ly in range(width):
        for lx in range(width):
            x, y = ix0 + lx, iy0 + ly
            r = lx + width * ly
            aw, ae = ax[y - 1, x - 1], ax[y - 1, x]
            as_, an = ay[y - 1, x - 1], ay[y, x - 1]
            A[r, r] = s * (kappa2 + (aw + ae + as_ + an) / h ** 2)
            for (nx, ny, a) in ((lx - 1, ly, aw), (lx + 1, ly, ae), (lx, ly - 1, as_), (lx, ly + 1, an)):
                if 0 <= nx < width and 0 <= ny < width:
                    A[r, nx + width * ny] = -s * a / h ** 2
    return A


def crop_prolongation(w, J0x, J0y, cw):
    """Dense P of a crop: coarse window J in [J0, J0+cw) per axis, fine window
    [2 J0 - 1, 2 (J0+cw-1) + 1]."""
    fw = 2 * cw + 1
    P = np.zeros((fw * fw, cw * cw))
    for ly in range(cw):
        for lx in range(cw):
            for t in range(9):
                dx, dy = t % 3 - 1, t // 3 - 1
                fx, fy = 2 * lx + 1 + dx, 2 * ly + 1 + dy
                P[fx + fw * fy, lx + cw * ly] = w[J0y + ly - 1, J0x + lx - 1, t]
    return P


def red_black_masks(ix0, iy0, width):
    """Sites of the window whose global coordinates have an even (red) or odd
    (black) coordinate sum; the forward sweep updates red first."""
    ly, lx = np.divmod(np.arange(width * width), width)
    red = ((lx + ix0 + ly + iy0) % 2) == 0
    return red, ~red


def gs_sweep(A, e, order):
    """Noise-free Gauss-Seidel sweep for A u = 0 from u = e, colour by colour
    (sites of one colour do not couple on the 5-point stencil)."""
    u = np.array(e, dtype=np.float64)  # a vector, or vectors as columns
    d = np.diag(A)
    for mask in order:
        dm = d[mask] if u.ndim == 1 else d[mask][:, None]
        u[mask] = u[mask] - (A[mask] @ u) / dm
    return u


def crop_loss_grad(faces, n, kappa2, w, errors, crops, cw=15, smooth=True):
    """Mean two-grid loss over crops x errors and its gradient w.r.t. w.
    errors: [K][n*n] fine vectors; crops: list of (J0x, J0y) coarse origins.
    smooth=False drops both smoothers (S_f = S_b = I)."""
    nc = (n - 1) // 2
    K = len(errors)
    dw = np.zeros_like(w)
    total = 0.0
    fw = 2 * cw + 1
    for (J0x, J0y) in crops:
        ix0, iy0 = 2 * J0x - 1, 2 * J0y - 1
        A = fine_operator_dense(faces, n, kappa2, ix0, iy0, fw)
        P = crop_prolongation(w, J0x, J0y, cw)
        Ac = P.T @ A @ P
        red, black = red_black_masks(ix0, iy0, fw)
        fwd, bwd = ((red, black), (black, red)) if smooth else ((), ())
        # S_b as a matrix: column j is the sweep of unit vector j
        Sb = gs_sweep(A, np.eye(fw * fw), bwd)
        W = Sb.T @ A @ Sb
        for e_full in errors:
            e = np.asarray(e_full, dtype=np.float64).reshape(n, n)[iy0 - 1:iy0 - 1 + fw, ix0 - 1:ix0 - 1 + fw].reshape(-1)
            E = e @ A @ e
            es = gs_sweep(A, e, fwd)
            x = np.linalg.solve(Ac, P.T @ (A @ es))
            r = es - P @ x
            total += (r @ W @ r) / E
            y = np.linalg.solve(Ac, P.T @ (W @ r))
            G = -2.0 * (np.outer(W @ r - A @ (P @ y), x) + np.outer(A @ r, y)) / E  # dL_e/dP
            for ly in range(cw):
                for lx in range(cw):
                    for t in range(9):
                        dx, dy = t % 3 - 1, t // 3 - 1
                        fx, fy = 2 * lx + 1 + dx, 2 * ly + 1 + dy
                        dw[J0y + ly - 1, J0x + lx - 1, t] += G[fx + fw * fy, lx + cw * ly]
    scale = 1.0 / (K * len(crops))
    return total * scale, dw * scale


def normalize_backward(o, nc, dw):
    """d loss / d o from d loss / d w through the normalisation and softplus."""
    rho = softplus(o)
    sig = 1.0 / (1.0 + np.exp(-o))
    drho = np.zeros_like(rho)
    w = normalize(o, nc)
    # fine node i collects the coarse nodes covering it; Z(i) = sum rho
    n_f = 2 * nc + 1
    for iy in range(1, n_f + 1):
        for ix in range(1, n_f + 1):
            if ix % 2 == 0 and iy % 2 == 0:
                continue
            cov = [(Ky, ey, Kx, ex) for Ky, ey in covering(iy, nc) for Kx, ex in covering(ix, nc)]
            Z = 0.0
            for Ky, ey, Kx, ex in cov:
                inside = 1 <= Kx <= nc and 1 <= Ky <= nc
                Z += rho[(ex + 1) + 3 * (ey + 1), Ky - 1, Kx - 1] if inside else 1.0
            s = 0.0
            for Ky, ey, Kx, ex in cov:
                if 1 <= Kx <= nc and 1 <= Ky <= nc:
                    t = (ex + 1) + 3 * (ey + 1)
                    s += dw[Ky - 1, Kx - 1, t] * w[Ky - 1, Kx - 1, t]
            for Ky, ey, Kx, ex in cov:
                if 1 <= Kx <= nc and 1 <= Ky <= nc:
                    t = (ex + 1) + 3 * (ey + 1)
                    drho[t, Ky - 1, Kx - 1] += (dw[Ky - 1, Kx - 1, t] - s) / Z
    drho[4] = 0.0
    return drho * sig


def loss_and_grad(theta, faces, n, kappa2, errors, crops, cw=15, smooth=True):
    """Loss of the network's prolongation and its gradient w.r.t. theta."""
    nc = (n - 1) // 2
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    X = features(faces, n)
    o, (X, z1, a1, z2, a2) = forward(theta, X)
    w = normalize(o, nc)
    loss, dw = crop_loss_grad(faces, n, kappa2, w, errors, crops, cw, smooth)
    do = normalize_backward(o, nc, dw)
    da2, dW3, db3 = conv3x3_backward(a2, W3, do)
    dz2 = da2 * (z2 > 0)
    da1, dW2, db2 = conv3x3_backward(a1, W2, dz2)
    dz1 = da1 * (z1 > 0)
    _, dW1, db1 = conv3x3_backward(X, W1, dz1)
    grad = np.concatenate([g.reshape(-1) for g in (dW1, db1, dW2, db2, dW3, db3)])
    return loss, grad


def init_params(seed):
    """Small random weights; the last bias makes softplus(b) = 1, i.e. the
    initial network reproduces multilinear interpolation up to the noise."""
    rng = np.random.default_rng(seed)
    out = []
    for s in SHAPES:
        if len(s) == 3:
            fan = s[1] * 9
            out.append(rng.normal(0.0, 1.0 / np.sqrt(fan), size=s) * (0.1 if s[0] == NOUT else 1.0))
        else:
            out.append(np.zeros(s))
    out[5][:] = np.log(np.expm1(1.0))
    return np.concatenate([a.reshape(-1) for a in out])
