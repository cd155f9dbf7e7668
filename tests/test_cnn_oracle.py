"""Pins of the CNN / cutout oracle (oracle/cnn.py) against facts outside it:
bf16 rounding by the float32 bit rule, a library cross-correlation, torch's
float64 layers and autograd, central finite differences, closed forms of the
loss and of Adam, brute-force pooling, and an identity that ties the two
cutout images together."""
import numpy as np
import pytest
import scipy.signal

import oracle
from oracle import cnn

RNG = np.random.default_rng(2110127495)


def rand_params(rng, scale=1.0):
    out = {}
    for name, shape in cnn.layout():
        if name.endswith(".w"):
            fan_in = int(np.prod(shape[1:])) if len(shape) > 1 else shape[0]
            out[name] = rng.uniform(-1, 1, shape) * np.sqrt(6.0 / fan_in) * scale
        else:
            out[name] = rng.normal(0, 0.05, shape)
    return cnn.pack(out)


# --- bf16 --------------------------------------------------------------------

def test_bf16_matches_float32_bit_rule():
    """For float32 inputs, rounding to 8 significant bits equals the usual
    bit rule on the float32 pattern: (u + 0x7FFF + ((u >> 16) & 1)) >> 16."""
    x = np.concatenate([RNG.normal(0, 1, 20000), RNG.normal(0, 1e-30, 2000), RNG.normal(0, 1e30, 2000)])
    x = x.astype(np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    bits = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    assert (cnn.bf16_bits(x.astype(np.float64)) == bits).all()


def test_bf16_ties_to_even():
    one = 1.0
    assert cnn.bf16(one + 2.0 ** -8) == 1.0                    # tie, 1.0 is even
    assert cnn.bf16(one + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6    # tie, rounds up to even
    assert cnn.bf16(one + 2.0 ** -8 + 2.0 ** -30) == 1.0 + 2.0 ** -7
    assert cnn.bf16(-(one + 3 * 2.0 ** -8)) == -(1.0 + 2.0 ** -6)
    assert cnn.bf16(2.0 ** -133 * 1.5) == 2.0 ** -132         # subnormal tie to even
    assert cnn.bf16(0.0) == 0.0


# --- layers --------------------------------------------------------------------

def test_conv3x3_equals_library_cross_correlation():
    x = RNG.normal(size=(2, 3, 7, 5))
    w = RNG.normal(size=(4, 3, 3, 3))
    b = RNG.normal(size=4)
    y = cnn.conv3x3(x, w, b)
    for n in range(2):
        for o in range(4):
            ref = b[o] + sum(scipy.signal.correlate2d(x[n, c], w[o, :, :, c], mode="same", boundary="fill")
                             for c in range(3))
            assert np.allclose(y[n, o], ref, rtol=1e-12, atol=1e-12)


def test_maxpool_first_maximum_and_routing_brute_force():
    a = RNG.integers(0, 3, size=(2, 3, 6, 4)).astype(np.float64)  # many ties
    p, q = cnn.maxpool2(a)
    dy = RNG.normal(size=p.shape)
    back = cnn.unpool2(dy, q, 6, 4)
    ref = np.zeros_like(a)
    for n in range(2):
        for c in range(3):
            for h in range(3):
                for w in range(2):
                    cells = [(2 * h, 2 * w), (2 * h, 2 * w + 1), (2 * h + 1, 2 * w), (2 * h + 1, 2 * w + 1)]
                    vals = [a[n, c, i, j] for i, j in cells]
                    k = vals.index(max(vals))
                    assert p[n, c, h, w] == max(vals) and q[n, c, h, w] == k
                    ref[n, c][cells[k]] = dy[n, c, h, w]
    assert (back == ref).all()


def test_bce_closed_forms():
    assert cnn.bce(0.0, 1.0) == pytest.approx(np.log(2.0), rel=1e-15)
    assert cnn.bce(0.0, 0.0) == pytest.approx(np.log(2.0), rel=1e-15)
    z = np.array([-30.0, -2.0, 0.5, 40.0])
    assert np.allclose(cnn.bce(z, 1.0), np.log1p(np.exp(-z)), rtol=1e-14)
    assert np.allclose(cnn.bce(z, 0.0), np.log1p(np.exp(z)), rtol=1e-14)


def test_adam_closed_forms():
    g = RNG.normal(size=50)
    p0 = RNG.normal(size=50)
    p1, m, v = cnn.adam(p0, g, np.zeros(50), np.zeros(50), 1, 1e-3)
    assert np.allclose(p1, p0 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    # a constant gradient keeps the bias-corrected moments at g and g^2
    p, m, v = p0, np.zeros(50), np.zeros(50)
    for t in range(1, 6):
        p, m, v = cnn.adam(p, g, m, v, t, 1e-3)
    assert np.allclose(p, p0 - 5e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-13)


# --- whole network ----------------------------------------------------------

@pytest.fixture(scope="module")
def net():
    rng = np.random.default_rng(7)
    p = rand_params(rng)
    x = rng.normal(size=(2, 2, 64, 64))
    y = np.array([1.0, 0.0])
    return p, x, y


def torch_reference(p, x, y):
    import torch
    import torch.nn.functional as F
    P = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in cnn.unpack(p).items()}
    a = torch.tensor(x, dtype=torch.float64)
    for l in range(4):
        w = P[f"conv{l + 1}.w"].permute(0, 3, 1, 2)  # [O][C][3][3]
        a = F.max_pool2d(F.relu(F.conv2d(a, w, P[f"conv{l + 1}.b"], padding=1)), 2)
    flat = a.permute(0, 2, 3, 1).reshape(a.shape[0], -1)
    h = F.relu(flat @ P["fc1.w"].T + P["fc1.b"])
    z = h @ P["fc2.w"] + P["fc2.b"]
    loss = F.binary_cross_entropy_with_logits(z, torch.tensor(y, dtype=torch.float64))
    loss.backward()
    g = np.concatenate([P[name].grad.numpy().reshape(-1) for name, _ in cnn.layout()])
    return z.detach().numpy(), float(loss), g


def test_parameter_count():
    assert cnn.num_params() == 490897


def test_forward_and_gradients_equal_torch_float64(net):
    """The float64 forward pass and its hand-written backward pass equal torch's
    float64 layers and autograd on the same parameters (torch routes a tied
    max-pool the same way only without ties: random inputs have none)."""
    p, x, y = net
    zt, lt, gt = torch_reference(p, x, y)
    z, _ = cnn.forward(p, x, quantized=False)
    g, l = cnn.gradients(p, x, y, quantized=False)
    assert np.allclose(z, zt, rtol=1e-12, atol=1e-12)
    assert l == pytest.approx(lt, rel=1e-12)
    for name, sl in slices():
        assert np.allclose(g[sl], gt[sl], rtol=1e-9, atol=1e-12 * np.abs(gt[sl]).max()), name


def slices():
    o = 0
    for name, shape in cnn.layout():
        n = int(np.prod(shape))
        yield name, slice(o, o + n)
        o += n


def test_gradients_equal_central_finite_differences(net):
    """Per parameter tensor, the directional derivative along a random
    direction equals the central difference of the float64 loss (relative
    error <= 1e-6), with the ReLU / pooling pattern unchanged across the
    difference."""
    p, x, y = net
    g, _ = cnn.gradients(p, x, y, quantized=False)
    base = cnn.pattern(p, x)
    rng = np.random.default_rng(11)
    for name, sl in slices():
        done = 0
        for attempt in range(6):
            v = np.zeros_like(p)
            v[sl] = rng.normal(size=sl.stop - sl.start)
            h = 1e-7 / np.sqrt(np.mean(v[sl] ** 2))
            if not ((cnn.pattern(p + h * v, x) == base).all() and (cnn.pattern(p - h * v, x) == base).all()):
                continue
            fd = (cnn.loss(p + h * v, x, y, quantized=False) - cnn.loss(p - h * v, x, y, quantized=False)) / (2 * h)
            an = float(g @ v)
            assert abs(fd - an) <= 1e-6 * abs(an) + 1e-12, (name, fd, an)
            done += 1
            if done == 2:
                break
        assert done >= 1, name


def test_quantized_network_is_the_float64_network_on_bf16_values(net):
    """quantized=True is the float64 network evaluated on the bf16-rounded
    input and weights (biases stay as given), nothing else rounded: equal to
    torch's float64 layers and autograd fed those rounded values, and a few
    bf16 steps away from the unrounded network."""
    p, x, y = net
    P = cnn.unpack(p)
    pq = cnn.pack({k: cnn.bf16(v) if k.endswith(".w") else v for k, v in P.items()})
    xq = cnn.bf16(x)
    zt, lt, gt = torch_reference(pq, xq, y)
    z, _ = cnn.forward(p, x, quantized=True)
    g, l = cnn.gradients(p, x, y, quantized=True)
    assert np.allclose(z, zt, rtol=1e-12, atol=1e-12)
    assert l == pytest.approx(lt, rel=1e-12)
    for name, sl in slices():
        assert np.allclose(g[sl], gt[sl], rtol=1e-9, atol=1e-12 * np.abs(gt[sl]).max()), name
    z0, _ = cnn.forward(p, x, quantized=False)
    assert np.abs(z - z0).max() <= 0.05 * (np.abs(z0).max() + 1e-3)


def test_layer_functions_compose_to_the_network(net):
    """Feeding each layer function the previous one's output (forward) and
    upstream gradient (backward) reproduces forward() and gradients()."""
    p, x, y = net
    P = cnn._params(p, True)
    a = cnn.bf16(x)
    ins, acts, qs = [], [], []
    for l in range(4):
        ins.append(a)
        act, a, q = cnn.conv_block(a, P[f"conv{l + 1}.w"], P[f"conv{l + 1}.b"])
        acts.append(act)
        qs.append(q)
    flat = cnn.flatten(a)
    h = cnn.fc1(flat, P["fc1.w"], P["fc1.b"])
    z = h @ P["fc2.w"] + P["fc2.b"][0]
    zf, _ = cnn.forward(p, x)
    assert np.array_equal(z, zf)
    dz, gw2, gb2, dh = cnn.head_backward(z, y, h, P["fc2.w"])
    gw1, gb1, dflat = cnn.fc1_backward(dh, flat, P["fc1.w"])
    G = {"fc2.w": gw2, "fc2.b": gb2, "fc1.w": gw1, "fc1.b": gb1}
    dy = dflat.reshape(-1, 4, 4, 128).transpose(0, 3, 1, 2)
    for l in range(3, -1, -1):
        G[f"conv{l + 1}.w"], G[f"conv{l + 1}.b"], dy, _ = cnn.conv_block_backward(
            dy, ins[l], P[f"conv{l + 1}.w"], acts[l], qs[l])
    g, _ = cnn.gradients(p, x, y)
    assert np.array_equal(cnn.pack(G), g)
    # dz closed form: sigmoid(z) - y over the batch
    assert np.allclose(dz, (1 / (1 + np.exp(-z)) - y) / len(y), rtol=1e-15)


def test_conv_block_input_gradient_is_the_transposed_convolution():
    """dx of a block equals torch's float64 autograd of the block's output
    against an arbitrary upstream gradient (the gradient the next layer
    down receives)."""
    import torch
    import torch.nn.functional as F
    rng = np.random.default_rng(13)
    x = rng.normal(size=(2, 5, 8, 8))
    w = rng.normal(size=(6, 3, 3, 5))
    b = rng.normal(size=6)
    act, pooled, q = cnn.conv_block(x, w, b)
    dp = rng.normal(size=pooled.shape)
    gw, gb, dx, _ = cnn.conv_block_backward(dp, x, w, act, q)
    xt = torch.tensor(x, requires_grad=True)
    wt = torch.tensor(w, requires_grad=True)
    bt = torch.tensor(b, requires_grad=True)
    out = F.max_pool2d(F.relu(F.conv2d(xt, wt.permute(0, 3, 1, 2), bt, padding=1)), 2)
    assert np.allclose(out.detach().numpy(), pooled, rtol=1e-13)
    out.backward(torch.tensor(dp))
    assert np.allclose(dx, xt.grad.numpy(), rtol=1e-12, atol=1e-12)
    assert np.allclose(gw, wt.grad.numpy(), rtol=1e-12, atol=1e-12)
    assert np.allclose(gb, bt.grad.numpy(), rtol=1e-12, atol=1e-12)


# --- cutouts -----------------------------------------------------------------

def cutout_inputs(nchan=128, nsamp=1500, D=1):
    rng = np.random.default_rng(5)
    freqs = 1000.0 + (np.arange(nchan) + 0.5) * 500.0 / nchan
    tsamp = 1e-3
    X = rng.integers(0, 256, size=(nsamp, nchan), dtype=np.uint8)
    seg = (0.0, 2.0, 70, D)
    row = oracle.dedisperse_segment(X, freqs, tsamp, seg)
    mu = np.array([oracle.stats(r)[0] for r in row])
    Y = oracle.downsample(X, D)
    delays = oracle.delay_table(freqs, tsamp, seg)
    return X, freqs, tsamp, seg, row, mu, Y, delays


def test_cutout_band_sum_equals_dm_time_line():
    """Without normalisation, the 64 sub-bands of the frequency-time image sum
    to the DM-time image's line of the candidate's trial (the dedispersed
    series is the channel sum), when no bin reaches before the data."""
    X, freqs, tsamp, seg, row, mu, Y, delays = cutout_inputs()
    for cand in [(40, 900, 24), (3, 700, 64), (69, 1100, 5)]:
        raw = cnn.cutout(row, mu, Y, delays, cand, normalize=False)
        lo = max(0, min(cand[0] - 32, row.shape[0] - 64))
        assert np.array_equal(raw[1].sum(axis=0), raw[0][cand[0] - lo])


def test_cutout_padding_and_normalisation():
    X, freqs, tsamp, seg, row, mu, Y, delays = cutout_inputs()
    cand = (10, 2, 40)  # e = 41, r = 5: bins before the data
    raw = cnn.cutout(row, mu, Y, delays, cand, normalize=False)
    # DM-time: bins wholly before the start are r * mean of their trial
    e, r = 41, 5
    for b in range(64):
        if e - (63 - b) * r < 0:
            assert np.allclose(raw[0][:, b], r * mu[:64])
    img = cnn.cutout(row, mu, Y, delays, cand)
    for k in range(2):
        assert abs(img[k].mean()) < 1e-12 and img[k].std() == pytest.approx(1.0, rel=1e-12)
    flat = cnn.cutout(np.full_like(row, 7), np.full(70, 7.0), np.full_like(Y, 3), delays, (20, 500, 8))
    assert (flat == 0).all()


def test_cutout_frequency_time_edge_rule_hand_computed():
    """A hand-computed case of the frequency-time edge rule: 64 channels, so
    each band is one channel; box end e = 116 and width 16 give bins of
    r = 2 samples starting at -11 + 2b.  Bin 5 covers samples -1 and 0 (one
    valid sample, scaled to two), bins 0..4 lie wholly before the data and
    take the mean of the band's 59 valid bins, bins 6..63 are plain sums of
    the channel's samples shifted by its delay."""
    nchan, N = 64, 300
    Y = (np.arange(nchan)[:, None] * 1000 + np.arange(N)[None, :] * 3 + (np.arange(N)[None, :] % 7)).astype(np.int64)
    delays = np.zeros((4, nchan), np.int64)
    delays[2] = np.arange(nchan) % 5
    row = np.zeros((4, N), np.int64)
    mu = np.zeros(4)
    raw = cnn.cutout(row, mu, Y, delays, (2, 101, 16), normalize=False)
    for j in range(nchan):
        d = int(delays[2, j])
        want = np.zeros(64)
        for b in range(6, 64):
            t0 = -11 + 2 * b
            want[b] = Y[j, t0 + d] + Y[j, t0 + 1 + d]
        want[5] = 2 * Y[j, 0 + d]
        want[:5] = want[5:].mean()
        assert np.allclose(raw[1][j], want, rtol=0, atol=1e-9), j
    # the same rule breaks visibly if the partial bin were left unscaled or
    # the empty bins left at zero
    assert raw[1][3][5] == 2 * Y[3, 3] and Y[3, 3] > 0
    assert raw[1][3][:5].min() > 0
