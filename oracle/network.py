"""Reference (FP64, numpy) for the proposal network of the learned block
move -- TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark baseline).

Network (gauge invariant in, coefficients out): per time slice t the input is
an 8-channel field on the spatial torus, the three spatial plaquettes of
slice t and of slice t+1 at each site (planes xy, xz, yz) and two zero
channels.  It never reads temporal links, so the proposal of a block never
depends on the links the block moves.  Three 3x3x3 periodic convolutions
(8 -> 32 -> 32 -> 32 channels, tanh) and a per-site linear head give six
numbers y[d] per site, one per block direction d = -x,+x,-y,+y,-z,+z.  The
block move uses c_d = beta r(a0_d)/sqrt(|S_d|^2+1) exp(y[d]) (see the
oracle's block move).  62502 parameters, one flat float vector in the order
W1[27][8][32], b1[32], W2[27][32][32], b2[32], W3[27][32][32], b3[32],
V[6][32], bv[6]; tap = (dz+1)*9 + (dy+1)*3 + (dx+1), and a convolution
reads input[s + (dx,dy,dz)].

Training loss: the negative mean log density of each site's temporal link
under its proposal, -mean log q(T | M), log q = (1/2)Tr(T M) - log Z(|M|),
over every site and slice of heat-bath configurations (maximum likelihood:
in equilibrium the link T(e) given everything except T(e) and its six
neighbours' temporal links follows the block marginal).

With `bf16=True` every operand of the convolution products (activations and
weights, forward and backward) is rounded to bfloat16 (round to nearest
even, from float32) and the products are summed in FP64; the GPU rounds the
same operands and sums in FP32.
"""
import numpy as np

from . import bessel_ive, block_pieces_all

CIN, CH, NTAP, NDIR = 8, 32, 27, 6
SHAPES = [("W1", (NTAP, CIN, CH)), ("b1", (CH,)), ("W2", (NTAP, CH, CH)), ("b2", (CH,)),
          ("W3", (NTAP, CH, CH)), ("b3", (CH,)), ("V", (NDIR, CH)), ("bv", (NDIR,))]
TAPS = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def param_count():
    return sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(params):
    out, off = {}, 0
    for name, shape in SHAPES:
        k = int(np.prod(shape))
        out[name] = np.asarray(params[off:off + k], dtype=np.float64).reshape(shape)
        off += k
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def init_params(seed):
    """Uniform(+-1/sqrt(fan_in)) weights, zero biases; the head starts at zero
    so that an untrained network proposes with the mean-field coefficients."""
    rng = np.random.default_rng(seed)
    d = {}
    for name, shape in SHAPES:
        if name.startswith("W"):
            fan = shape[0] * shape[1]
            d[name] = rng.uniform(-1, 1, size=shape) / np.sqrt(fan)
        else:
            d[name] = np.zeros(shape)
    d["V"] = np.zeros((NDIR, CH))
    return pack(d).astype(np.float32).astype(np.float64)


def bf16(x):
    """Round to bfloat16 (nearest even) via float32, returned as float64."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) >> 16 << 16
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def _r(x, on):
    return bf16(x) if on else np.asarray(x, dtype=np.float64)


def _qmul(a, b):
    a0, a1, a2, a3 = np.moveaxis(a, -1, 0)
    b0, b1, b2, b3 = np.moveaxis(b, -1, 0)
    return np.stack([a0 * b0 - a1 * b1 - a2 * b2 - a3 * b3,
                     a0 * b1 + b0 * a1 - a2 * b3 + a3 * b2,
                     a0 * b2 + b0 * a2 - a3 * b1 + a1 * b3,
                     a0 * b3 + b0 * a3 - a1 * b2 + a2 * b1], -1)


def _dag(a):
    return a * np.array([1.0, -1.0, -1.0, -1.0])


def _shift(a, dx, dy, dz):
    """b[t, z, y, x] = a[t, z + dz, y + dy, x + dx] (periodic)."""
    return np.roll(a, shift=(-dz, -dy, -dx), axis=(1, 2, 3))


def features(n, U):
    """(Nt, Nz, Ny, Nx, 8): spatial plaquettes of slices t and t+1, two zeros."""
    nt = n[3]
    F = np.zeros((nt, n[2], n[1], n[0], CIN))
    axes = {0: (1, 0, 0), 1: (0, 1, 0), 2: (0, 0, 1)}
    for c, (i, j) in enumerate([(0, 1), (0, 2), (1, 2)]):
        Ui, Uj = U[..., i, :], U[..., j, :]
        Uj_i = _shift(Uj, *axes[i])
        Ui_j = _shift(Ui, *axes[j])
        p = _qmul(_qmul(Ui, Uj_i), _qmul(_dag(Ui_j), _dag(Uj)))[..., 0]
        F[..., c] = p
        F[..., 3 + c] = np.roll(p, -1, axis=0)
    return F


def conv3(a, W, b, rnd):
    out = np.broadcast_to(b, a.shape[:-1] + (W.shape[2],)).copy()
    Wr = _r(W, rnd)
    for tap, (dx, dy, dz) in enumerate(TAPS):
        out += _r(_shift(a, dx, dy, dz), rnd) @ Wr[tap]
    return out


def forward(feat, params, rnd=True):
    p = unpack(params)
    a1 = np.tanh(conv3(feat, p["W1"], p["b1"], rnd))
    a2 = np.tanh(conv3(a1, p["W2"], p["b2"], rnd))
    a3 = np.tanh(conv3(a2, p["W3"], p["b3"], rnd))
    y = a3 @ p["V"].T + p["bv"]
    return {"feat": feat, "a1": a1, "a2": a2, "a3": a3, "y": y}


def log_z(a):
    a = np.asarray(a, dtype=np.float64)
    out = np.zeros_like(a)
    nz = a > 0
    out[nz] = np.log(2 * np.vectorize(lambda x: bessel_ive(1, x))(a[nz]) / a[nz]) + a[nz]
    return out


def bessel_ratio(a):
    a = np.asarray(a, dtype=np.float64)
    out = np.zeros_like(a)
    nz = a > 0
    out[nz] = (np.vectorize(lambda x: bessel_ive(2, x))(a[nz]) /
               np.vectorize(lambda x: bessel_ive(1, x))(a[nz]))
    return out


def proposal_coefficients(S, y, beta):
    """c[..., d] = beta r(a0)/sqrt(|S_d|^2+1) exp(y_d), a0 = beta sqrt(|S_d|^2+1)."""
    s2 = (S * S).sum(-1)
    root = np.sqrt(s2 + 1.0)
    return beta * bessel_ratio(beta * root) / root * np.exp(y)


def loss_and_grad_y(n, U, y, beta, S=None):
    """Mean negative log proposal density of every temporal link, and its
    gradient with respect to the network outputs y (same shape as y)."""
    if S is None:
        S = block_pieces_all(n, U)
    c = proposal_coefficients(S, y, beta)
    M = (c[..., None] * S).sum(-2)
    k = np.sqrt((M * M).sum(-1))
    T = U[..., 3, :]
    htm = _qmul(T, M)[..., 0]
    logq = htm - log_z(k)
    N = logq.size
    loss = -logq.mean()
    # d/dc_d [ (1/2)Tr(T M) - log Z(|M|) ] = (1/2)Tr(T S_d) - r(|M|) <Mhat, S_d>
    hts = _qmul(np.broadcast_to(T[..., None, :], S.shape), S)[..., 0]
    Mhat = np.where(k[..., None] > 0, M / np.maximum(k, 1e-300)[..., None], 0.0)
    dots = (Mhat[..., None, :] * S).sum(-1)
    dlogq_dc = hts - bessel_ratio(k)[..., None] * dots
    dy = -(dlogq_dc * c) / N
    return loss, dy


def backward(cache, dy, params, rnd=True):
    """Gradient of the loss with respect to the flat parameter vector, given
    dL/dy; rounding points as on the GPU."""
    p = unpack(params)
    feat, a1, a2, a3 = cache["feat"], cache["a1"], cache["a2"], cache["a3"]
    g = {}
    g["V"] = dy.reshape(-1, NDIR).T @ a3.reshape(-1, CH)
    g["bv"] = dy.reshape(-1, NDIR).sum(0)
    da = dy @ p["V"]
    for layer, a_in, a_out in ((3, a2, a3), (2, a1, a2), (1, feat, a1)):
        dz = da * (1.0 - a_out * a_out)
        W = p[f"W{layer}"]
        dzr = _r(dz, rnd)
        gW = np.zeros_like(W)
        for tap, (dx, dy_, dz_) in enumerate(TAPS):
            gW[tap] = _r(_shift(a_in, dx, dy_, dz_), rnd).reshape(-1, W.shape[1]).T @ dzr.reshape(-1, W.shape[2])
        g[f"W{layer}"] = gW
        g[f"b{layer}"] = dz.reshape(-1, W.shape[2]).sum(0)
        if layer > 1:
            Wr = _r(W, rnd)
            da = np.zeros_like(a_in)
            for tap, (dx, dy_, dz_) in enumerate(TAPS):
                da += _shift(dzr, -dx, -dy_, -dz_) @ Wr[tap].T
    return pack(g)


def adam(params, grad, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (step counts from 1); returns new (params, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
