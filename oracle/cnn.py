"""CPU oracle of candidate cutouts and of the triage network (numpy, float64).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use this module.  It shares no code with
the GPU library and imports nothing from it.

The paper names the classification of candidates as a pipeline stage
(Section 2.1) and the candidates' way into the database (Section 4) but fixes
no classifier, no cutout and no training recipe: parity unpinned by the
paper.  What is computed here is the plain definition of the network and
cutouts declared in the library's header, pinned by mathematics instead:
central finite differences of the loss, torch's float64 layers and autograd,
a library cross-correlation for the convolutions, closed forms of the loss,
of Adam's first steps and of the pooling routing, brute-force loops on tiny
inputs.

The network is defined on bf16 numbers: its input images and its weights
are bf16 values.  ``quantized=True`` rounds the given input and weights to
bf16 (nearest even) and then computes every product, sum and nonlinearity
of the forward and backward passes in float64, with no further rounding;
``quantized=False`` rounds nothing (a smooth function of the parameters
between ReLU / max-pool pattern changes, the one the finite-difference pins
check).  Where an implementation stores an intermediate result at lower
precision, its tests compare that stored value with the float64 one here.
The layer functions (``conv_block``, ``conv_block_backward``, ``fc1``,
``fc1_backward``, ``head_backward``) take their inputs explicitly so that a
test can feed each layer the implementation's own stored input or upstream
gradient.
"""
from __future__ import annotations

import numpy as np

CONV = [(2, 16, 64), (16, 32, 32), (32, 64, 16), (64, 128, 8)]  # (cin, cout, input height = width)
FLAT = 128 * 4 * 4
HIDDEN = 192


def bf16(x):
    """Round to the nearest bf16 value (8 significant bits, ties to even;
    subnormals are multiples of 2**-133), returned as float64."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)
    normal = np.ldexp(np.rint(np.ldexp(m, 8)), e - 8)
    sub = np.ldexp(np.rint(np.ldexp(x, 133)), -133)
    return np.where(e >= -125, normal, sub)


def bf16_bits(x):
    """uint16 bit patterns of bf16(x) (for feeding the GPU)."""
    v = bf16(x).astype(np.float32)
    return (v.view(np.uint32) >> 16).astype(np.uint16)


def from_bf16_bits(b):
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def layout():
    """[(name, shape)] of the parameter vector, in order."""
    out = []
    for l, (ci, co, _) in enumerate(CONV):
        out += [(f"conv{l + 1}.w", (co, 3, 3, ci)), (f"conv{l + 1}.b", (co,))]
    out += [("fc1.w", (HIDDEN, FLAT)), ("fc1.b", (HIDDEN,)), ("fc2.w", (HIDDEN,)), ("fc2.b", (1,))]
    return out


def num_params():
    return int(sum(np.prod(s) for _, s in layout()))


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    out, o = {}, 0
    for name, shape in layout():
        n = int(np.prod(shape))
        out[name] = p[o:o + n].reshape(shape)
        o += n
    assert o == p.size
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in layout()])


def conv3x3(x, w, b):
    """y[n,o,h,v] = b[o] + sum_{c,i,j} w[o,i,j,c] x[n,c,h+i-1,v+j-1] (zero padding 1).
    x [N][C][H][W], w [O][3][3][C]."""
    N, C, H, W = x.shape
    xp = np.zeros((N, C, H + 2, W + 2))
    xp[:, :, 1:-1, 1:-1] = x
    y = np.zeros((N, w.shape[0], H, W)) + b[None, :, None, None]
    for i in range(3):
        for j in range(3):
            y += np.einsum("nchw,oc->nohw", xp[:, :, i:i + H, j:j + W], w[:, i, j, :], optimize=True)
    return y


def maxpool2(a):
    """2x2 max-pool; index q = 2*(row parity) + (column parity) of the first maximum."""
    N, C, H, W = a.shape
    win = a.reshape(N, C, H // 2, 2, W // 2, 2).transpose(0, 1, 2, 4, 3, 5).reshape(N, C, H // 2, W // 2, 4)
    q = np.argmax(win, axis=-1)
    return np.take_along_axis(win, q[..., None], axis=-1)[..., 0], q


def unpool2(dy, q, H, W):
    """Route dy [N][C][H/2][W/2] to the pooled positions q (inverse of maxpool2's gather)."""
    N, C = dy.shape[:2]
    out = np.zeros((N, C, H // 2, W // 2, 4))
    np.put_along_axis(out, q[..., None], dy[..., None], axis=-1)
    return out.reshape(N, C, H // 2, W // 2, 2, 2).transpose(0, 1, 2, 4, 3, 5).reshape(N, C, H, W)


def conv_block(x, w, b):
    """One convolution block: act = ReLU(conv3x3(x, w) + b), then a 2x2
    max-pool.  Returns (act [N][O][H][W], pooled [N][O][H/2][W/2], q)."""
    act = np.maximum(conv3x3(x, w, b), 0.0)
    pooled, q = maxpool2(act)
    return act, pooled, q


def conv_block_backward(dpooled, x, w, act, q):
    """Gradients of one block given the gradient of its pooled output:
    dpre = (dpooled routed to the pooled positions q) * [act > 0];
    dW[o,i,j,c] = sum_{n,h,v} dpre[n,o,h,v] x[n,c,h+i-1,v+j-1];
    db[o] = sum dpre[n,o,h,v];
    dx[n,c,h,v] = sum_{o,i,j} dpre[n,o,h-i+1,v-j+1] w[o,i,j,c].
    Returns (dW, db, dx, dpre)."""
    n, ci, H, _ = x.shape
    dpre = unpool2(dpooled, q, H, H) * (act > 0)
    xp = np.zeros((n, ci, H + 2, H + 2))
    xp[:, :, 1:-1, 1:-1] = x
    gw = np.zeros((w.shape[0], 3, 3, ci))
    dxp = np.zeros((n, ci, H + 2, H + 2))
    for i in range(3):
        for j in range(3):
            gw[:, i, j, :] = np.einsum("nohw,nchw->oc", dpre, xp[:, :, i:i + H, j:j + H], optimize=True)
            dxp[:, :, i:i + H, j:j + H] += np.einsum("nohw,oc->nchw", dpre, w[:, i, j, :], optimize=True)
    return gw, dpre.sum(axis=(0, 2, 3)), dxp[:, :, 1:-1, 1:-1], dpre


def flatten(pooled):
    """[N][128][4][4] -> [N][2048] in (h, w, c) order."""
    return pooled.transpose(0, 2, 3, 1).reshape(pooled.shape[0], FLAT)


def fc1(flat, w, b):
    """Hidden layer h = ReLU(flat w^T + b)."""
    return np.maximum(flat @ w.T + b, 0.0)


def head_backward(z, y, h, w2):
    """Loss head: mean BCE over the batch of z = h w2 + b2.  Returns
    (dz = (sigmoid(z) - y) / n, dW2 = dz h, db2 = sum dz,
    dh = dz w2 * [h > 0], the gradient of fc1's pre-activation)."""
    n = z.shape[0]
    dz = (1.0 / (1.0 + np.exp(-z)) - y) / n
    return dz, dz @ h, np.array([dz.sum()]), np.outer(dz, w2) * (h > 0)


def fc1_backward(dh, flat, w1):
    """Given the gradient dh of fc1's pre-activation: (dW1 = dh^T flat,
    db1 = sum_n dh, dflat = dh w1)."""
    return dh.T @ flat, dh.sum(axis=0), dh @ w1


def _params(params, quantized):
    r = bf16 if quantized else (lambda a: a)
    return {k: r(v) if k.endswith(".w") else v for k, v in unpack(params).items()}


def forward(params, x, quantized=True):
    """x: [N][2][64][64].  Returns (logits [N], cache)."""
    P = _params(params, quantized)
    a = bf16(np.asarray(x, dtype=np.float64)) if quantized else np.asarray(x, dtype=np.float64)
    cache = {"P": P, "in": [], "act": [], "q": []}
    for l in range(4):
        cache["in"].append(a)
        act, a, q = conv_block(a, P[f"conv{l + 1}.w"], P[f"conv{l + 1}.b"])
        cache["act"].append(act)
        cache["q"].append(q)
    cache["pooled"] = a
    flat = flatten(a)
    h = fc1(flat, P["fc1.w"], P["fc1.b"])
    z = h @ P["fc2.w"] + P["fc2.b"][0]
    cache.update(flat=flat, h=h, z=z)
    return z, cache


def bce(z, y):
    """Per-sample binary cross-entropy of logits z against labels y."""
    z = np.asarray(z, dtype=np.float64)
    return np.maximum(z, 0.0) - z * y + np.log1p(np.exp(-np.abs(z)))


def loss(params, x, y, quantized=True):
    z, _ = forward(params, x, quantized)
    return float(np.mean(bce(z, y)))


def pattern(params, x):
    """ReLU signs and pooling choices of the unrounded forward pass (the loss
    is smooth in the parameters while this stays the same)."""
    _, c = forward(params, x, quantized=False)
    parts = [(a > 0).ravel() for a in c["act"]] + [q.ravel() for q in c["q"]] + [(c["h"] > 0).ravel()]
    return np.concatenate([p.astype(np.int64) for p in parts])


def gradients(params, x, y, quantized=True):
    """Gradient of the mean loss with respect to the parameter vector; (grad, loss)."""
    z, c = forward(params, x, quantized)
    P = c["P"]
    y = np.asarray(y, dtype=np.float64)
    G = {}
    _, G["fc2.w"], G["fc2.b"], dh = head_backward(z, y, c["h"], P["fc2.w"])
    G["fc1.w"], G["fc1.b"], dflat = fc1_backward(dh, c["flat"], P["fc1.w"])
    dy = dflat.reshape(-1, 4, 4, 128).transpose(0, 3, 1, 2)
    for l in range(3, -1, -1):
        G[f"conv{l + 1}.w"], G[f"conv{l + 1}.b"], dy, _ = conv_block_backward(
            dy, c["in"][l], P[f"conv{l + 1}.w"], c["act"][l], c["q"][l])
    return pack(G), float(np.mean(bce(z, y)))


def adam(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba, ICLR 2015, Algorithm 1) at step t >= 1;
    returns (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


# ---------------------------------------------------------------------------
# cutouts
# ---------------------------------------------------------------------------
def cutout(dmt_row, mu_row, Y, delays, cand, rmax=8, normalize=True):
    """The two images of one candidate, z-scored, float64 (bf16 is applied by
    the caller).
    dmt_row: int [n_dm][n_out] dedispersed series of the candidate's row;
    mu_row: float [n_dm] their means; Y: int [nchan][N] the row's
    downsampled input (channel-major); delays: int [n_dm][nchan] the row's
    delay table; cand: (dm_index, t_peak, width)."""
    i, t_peak, w = (int(v) for v in cand)
    n_dm, n_out = dmt_row.shape
    nchan = Y.shape[0]
    e = t_peak + w - 1
    r = max(1, min(rmax, w // 8))
    lo = max(0, min(i - 32, n_dm - 64))
    starts = [e - (64 - b) * r + 1 for b in range(64)]
    dmimg = np.zeros((64, 64))
    for q in range(64):
        tr = lo + q
        if tr >= n_dm:
            continue
        for b, t0 in enumerate(starts):
            s = 0.0
            for t in range(t0, t0 + r):
                s += float(dmt_row[tr, t]) if t >= 0 else mu_row[tr]
            dmimg[q, b] = s
    ftimg = np.zeros((64, 64))
    for j in range(64):
        chans = range(j * nchan // 64, (j + 1) * nchan // 64)
        valid = []
        for b, t0 in enumerate(starts):
            ts = [t for t in range(t0, t0 + r) if t >= 0]
            if not ts:
                ftimg[j, b] = np.nan
                continue
            s = 0
            for ch in chans:
                d = int(delays[i, ch])
                s += int(sum(int(Y[ch, t + d]) for t in ts))
            ftimg[j, b] = s * r / len(ts)
            valid.append(ftimg[j, b])
        if len(valid) < 64:
            fill = float(np.mean(valid)) if valid else 0.0
            ftimg[j][np.isnan(ftimg[j])] = fill
    if not normalize:
        return np.stack([dmimg, ftimg])
    out = []
    for img in (dmimg, ftimg):
        if img.min() == img.max():
            out.append(np.zeros_like(img))
        else:
            mean = img.mean()
            out.append((img - mean) / np.sqrt(np.mean((img - mean) ** 2)))
    return np.stack(out)
