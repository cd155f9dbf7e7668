"""Triage network and cutouts on the GPU against the CPU oracle (oracle/cnn.py).

Per layer, the oracle is fed the GPU's own bf16 input to that layer, so a
difference can only come from the layer itself: float32 vs float64
accumulation moves a stored bf16 value by at most one rounding step.  End to
end (logits, gradients) the oracle starts from the same bf16 input and
parameters, and rounding steps that fall differently propagate; the bound
there is looser and stated per test."""
import numpy as np
import pytest

import oracle
from oracle import cnn as ocnn
from paper_2110_12749_amd import synth
from tests._util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env(dev):
    import torch
    from paper_2110_12749_amd import gsp
    ctx = gsp.Context(0)
    yield gsp, ctx, torch
    torch.cuda.synchronize()
    ctx.close()


def to_dev(torch, x):
    """float64 values -> bf16 bit patterns on the device (torch.int16)."""
    return torch.from_numpy(ocnn.bf16_bits(x).view(np.int16)).to("cuda:0")


def inputs(n, seed):
    rng = np.random.default_rng(seed)
    x = ocnn.bf16(rng.normal(size=(n, 2, 64, 64)))
    y = (rng.random(n) < 0.5).astype(np.float64)
    return x, y


def close_bf16(gpu, ora, what):
    """bf16-stored values: equal up to one rounding step (relative 2^-7 of the
    larger magnitude, or a tiny absolute amount near 0), mostly identical."""
    scale = np.abs(ora).max() + 1e-30
    diff = np.abs(gpu - ora)
    bound = 2.0 ** -7 * np.maximum(np.abs(gpu), np.abs(ora)) + 1e-5 * scale
    bad = diff > bound
    same = np.mean(gpu == ora)
    say(f"  {what}: identical {same:.5f}, max rel diff {np.max(diff / (np.abs(ora) + 1e-3 * scale)):.2e}")
    assert not bad.any(), (what, np.argwhere(bad)[:5], gpu[bad][:5], ora[bad][:5])
    assert same >= 0.98, (what, same)


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / (np.linalg.norm(b) + 1e-30))


def nchw(a):
    return a.transpose(0, 3, 1, 2)


def test_forward_layer_by_layer(env):
    gsp, ctx, torch = env
    net = gsp.Cnn(ctx, seed=3)
    p = net.params().astype(np.float64)
    P = {k: (ocnn.bf16(v) if k.endswith(".w") else v) for k, v in ocnn.unpack(p).items()}
    for n in (1, 5, 37):  # 37: a ragged GEMM tail in M for every layer
        say(f"[case] forward layers, batch {n}")
        x, _ = inputs(n, 100 + n)
        z = net.forward(to_dev(torch, x)).cpu().numpy()
        a = x
        for l in range(4):
            act_ref, _, _ = ocnn.conv_block(a, P[f"conv{l + 1}.w"], P[f"conv{l + 1}.b"])
            act = nchw(net.activation(12 + l, n))
            close_bf16(act, ocnn.bf16(act_ref), f"conv{l + 1} ReLU output")
            # pooling of the stored bf16 activations: exact values and choices
            pooled_ref, q_ref = ocnn.maxpool2(act)
            got = nchw(net.activation(l, n))
            assert np.array_equal(got, pooled_ref), l
            assert np.array_equal(nchw(net.activation(16 + l, n)).astype(np.int64), q_ref), l
            a = got  # next layer from the GPU's own input
        flat = ocnn.flatten(a)
        href = ocnn.fc1(flat, P["fc1.w"], P["fc1.b"])
        h = net.activation(4, n)
        close_bf16(h, ocnn.bf16(href), "fc1")
        zref = h @ P["fc2.w"] + P["fc2.b"][0]
        mag = np.abs(h) @ np.abs(P["fc2.w"]) + abs(P["fc2.b"][0])
        assert np.all(np.abs(z - zref) <= 1e-5 * mag + 1e-6), (z, zref)
        assert np.array_equal(net.activation(5, n), z)
        # end to end from the same input against the float64 network: a
        # stored value that rounds the other way moves the logits by a few
        # bf16 steps of their scale
        zo, _ = ocnn.forward(p, x)
        dz = np.abs(z - zo).max() / (np.abs(zo).max() + 1e-3)
        say(f"  logits end to end: max diff / scale {dz:.2e}")
        assert dz <= 0.05
    net.close()


def fp32_kept(got, ref, what, errs):
    e = rel_l2(got, ref)
    errs[what] = e
    say(f"  {what}: rel L2 {e:.2e}")
    assert e <= 1e-3, (what, e)


def test_gradients_layer_by_layer(env):
    """Every layer of the backward pass fed the GPU's own stored forward
    tensors and upstream gradient: parameter gradients (kept in fp32) within
    relative L2 1e-3 of the float64 definition, stored bf16 gradients within
    one bf16 rounding step (2^-7 relative) of it."""
    gsp, ctx, torch = env
    net = gsp.Cnn(ctx, seed=4)
    p = net.params().astype(np.float64)
    P = {k: (ocnn.bf16(v) if k.endswith(".w") else v) for k, v in ocnn.unpack(p).items()}
    for n in (3, 16, 37):
        say(f"[case] gradients, batch {n}")
        x, y = inputs(n, 200 + n)
        g, loss = net.gradients(to_dev(torch, x), torch.from_numpy(y.astype(np.float32)).cuda())
        G = ocnn.unpack(g.astype(np.float64))
        errs = {}
        # loss head, fed the GPU's logits and hidden layer
        z = net.activation(5, n).astype(np.float64)
        h = net.activation(4, n)
        dz, dw2, db2, dh = ocnn.head_backward(z, y, h, P["fc2.w"])
        assert loss == pytest.approx(float(np.mean(ocnn.bce(z, y))), rel=1e-5)
        dz_gpu = net.activation(11, n).astype(np.float64)
        assert np.all(np.abs(dz_gpu - dz) <= 1e-5 * np.abs(dz) + 1e-7 / n), (dz_gpu, dz)
        fp32_kept(G["fc2.w"], dw2, "fc2.w", errs)
        fp32_kept(G["fc2.b"], db2, "fc2.b", errs)
        dh_gpu = net.activation(10, n)
        close_bf16(dh_gpu, ocnn.bf16(dh), "d fc1 pre-activation")
        # fc1, fed the GPU's upstream gradient and input
        flat = ocnn.flatten(nchw(net.activation(3, n)))
        dw1, db1, dflat = ocnn.fc1_backward(dh_gpu, flat, P["fc1.w"])
        fp32_kept(G["fc1.w"], dw1, "fc1.w", errs)
        fp32_kept(G["fc1.b"], db1, "fc1.b", errs)
        dpool3 = net.activation(9, n).reshape(n, -1)
        close_bf16(dpool3, ocnn.bf16(dflat), "d pooled output of block 4")
        # convolution blocks, each fed the GPU's gradient of its pooled output
        for l in range(3, -1, -1):
            dy = nchw(net.activation(6 + l, n))
            xin = x if l == 0 else nchw(net.activation(l - 1, n))
            act = nchw(net.activation(12 + l, n))
            q = nchw(net.activation(16 + l, n)).astype(np.int64)
            gw, gb, dx, _ = ocnn.conv_block_backward(dy, xin, P[f"conv{l + 1}.w"], act, q)
            fp32_kept(G[f"conv{l + 1}.w"], gw, f"conv{l + 1}.w", errs)
            fp32_kept(G[f"conv{l + 1}.b"], gb, f"conv{l + 1}.b", errs)
            if l > 0:
                close_bf16(nchw(net.activation(6 + l - 1, n)), ocnn.bf16(dx), f"d pooled output of block {l}")
        # end to end against the float64 network on the same bf16 input and
        # weights: stored activations and gradients rounding the other way
        # propagate, so the bound is looser than per layer
        ge, le = ocnn.gradients(p, x, y)
        e2e = rel_l2(g.astype(np.float64), ge)
        say(f"  whole gradient vs float64 network: rel L2 {e2e:.2e}; loss {loss:.6f} vs {le:.6f}")
        assert e2e <= 0.05
        assert loss == pytest.approx(le, rel=1e-2)
    net.close()


def test_train_step_is_adam_on_the_gradients(env):
    gsp, ctx, torch = env
    net = gsp.Cnn(ctx, seed=5)
    x, y = inputs(8, 300)
    xd, yd = to_dev(torch, x), torch.from_numpy(y.astype(np.float32)).cuda()
    lr = 1e-3
    p = net.params().astype(np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    for t in (1, 2, 3):
        g, _ = net.gradients(xd, yd)
        g = g.astype(np.float64)
        net.train_step(xd, yd, lr)
        got = net.params().astype(np.float64)
        p, m, v = ocnn.adam(p, g, m, v, t, lr)
        # train_step recomputes the gradient (atomic split-K sums: last-bit
        # differences), so elements whose gradient nearly cancels are excluded
        sig = np.abs(g) > 1e-4 * np.abs(g).max()
        err = np.abs(got - p)
        ok = err <= 2e-3 * lr + 2.0 ** -22 * np.abs(p)
        say(f"  step {t}: significant {sig.mean():.3f}, matching {ok[sig].mean():.5f}, max err {err[sig].max():.2e}")
        assert ok[sig].mean() >= 0.999
        p = got  # continue from the GPU's parameters
    net.close()


def test_training_learns_a_separable_task(env):
    gsp, ctx, torch = env
    net = gsp.Cnn(ctx, seed=6)
    rng = np.random.default_rng(400)

    def batch(n):
        y = (rng.random(n) < 0.5).astype(np.float32)
        x = rng.normal(size=(n, 2, 64, 64))
        x[y == 1, 0, 28:36, 56:64] += 2.0  # a bright patch in the DM-time image
        return to_dev(torch, x), torch.from_numpy(y).cuda()

    losses = []
    for it in range(60):
        xd, yd = batch(64)
        losses.append(net.train_step(xd, yd, 1e-3))
    xd, yd = batch(256)
    z = net.forward(xd).cpu().numpy()
    acc = np.mean((z > 0) == (yd.cpu().numpy() > 0.5))
    say(f"  loss {losses[0]:.3f} -> {np.mean(losses[-5:]):.3f}, held-out accuracy {acc:.3f}")
    assert np.mean(losses[-5:]) < 0.5 * losses[0]
    assert acc >= 0.95
    net.close()


def test_save_load_roundtrip(env, tmp_path):
    gsp, ctx, torch = env
    a = gsp.Cnn(ctx, seed=7)
    b = gsp.Cnn(ctx, seed=8)
    assert not np.array_equal(a.params(), b.params())
    a.save(str(tmp_path / "w.bin"))
    b.load(str(tmp_path / "w.bin"))
    assert np.array_equal(a.params(), b.params())
    x, _ = inputs(4, 500)
    xd = to_dev(torch, x)
    assert torch.equal(a.forward(xd), b.forward(xd))
    a.close()
    b.close()


# --- cutouts -------------------------------------------------------------------

def cutout_case(env, w, extra, batch=0, check=None):
    """GPU cutouts of the search's candidates plus `extra` (seg, dm_index,
    t_peak, width) against the oracle, bf16 bit for bit up to rare one-step
    rounding differences.  batch > 0: random valid candidates are added up to
    that many (a batch large enough for the channel-major path) and the
    oracle checks the candidates listed in `check` (default: all)."""
    gsp, ctx, torch = env
    X = w.generate()
    fb = torch.from_numpy(X).cuda()
    desc = gsp.plan_shape(w.nsamp, w.freqs, w.tsamp, w.segments)
    dmt = ctx.dedisperse(fb, w.freqs, desc)
    c = ctx.single_pulse_search(dmt, desc, w.widths, w.threshold)
    c = c[np.argsort(-c["snr"])][:12]
    more = np.zeros(len(extra), c.dtype)
    for k, (s, i, t, wd) in enumerate(extra):
        more[k]["seg"], more[k]["dm_index"], more[k]["t_peak"], more[k]["width"] = s, i, t, wd
    c = np.concatenate([c, more])
    if batch > len(c):
        rng = np.random.default_rng(5)
        fill = np.zeros(batch - len(c), c.dtype)
        fill["seg"] = rng.integers(0, desc.n_seg, len(fill))
        for k in range(len(fill)):
            s = int(fill[k]["seg"])
            wd = int(rng.choice(w.widths))
            fill[k]["dm_index"] = rng.integers(0, desc.seg[s].n_dm)
            fill[k]["width"] = wd
            fill[k]["t_peak"] = rng.integers(0, desc.n_out[s] - wd + 1)
        c = np.concatenate([c, fill])
    say(f"[case] cutouts {w.name}: {len(c)} candidates, widths {sorted(set(c['width'].tolist()))}")
    out = gsp.cutouts(ctx, fb, w.freqs, dmt, desc, c).cpu().numpy().view(np.uint16)
    rows = oracle.dedisperse(X, w.freqs, w.tsamp, w.segments)
    per_row = {}
    total_px, diff_px = 0, 0
    for k in (range(len(c)) if check is None else check):
        cand = c[k]
        s = int(cand["seg"])
        if s not in per_row:
            seg = w.segments[s]
            per_row[s] = (rows[s], np.array([oracle.stats(r)[0] for r in rows[s]]), oracle.downsample(X, seg[3]),
                          oracle.delay_table(w.freqs, w.tsamp, seg))
        row, mu, Y, delays = per_row[s]
        ref = ocnn.bf16_bits(ocnn.cutout(row, mu, Y, delays, (cand["dm_index"], cand["t_peak"], cand["width"])))
        got = out[k]
        g = ocnn.from_bf16_bits(got)
        r = ocnn.from_bf16_bits(ref)
        assert np.all(np.abs(g - r) <= 2.0 ** -7 * np.maximum(np.abs(g), np.abs(r)) + 1e-6), k
        total_px += got.size
        diff_px += int(np.sum(got != ref))
    say(f"  pixels differing by one rounding step: {diff_px} of {total_px}")
    assert diff_px <= 1e-3 * total_px


def test_cutouts_tiny(env):
    w = synth.tiny()
    # near the start (bins before the data), near the end, edge trials, widths up to r = 8
    cutout_case(env, w, [(0, 0, 0, 1), (0, 5, 3, 40), (0, 199, 14072 - 64, 64), (0, 100, 500, 17),
                         (0, 57, 7000, 200)])


def test_cutouts_multirow(env):
    segs = [(0.0, 1.0, 40, 1), (40.0, 2.0, 70, 2), (180.0, 4.0, 12, 4)]
    w = synth.small(nchan=192, nsamp=6000, segments=segs, n_pulses=3, seed_offset=60, widths=[1, 2, 4, 8, 16, 32])
    desc_rows = [(1, 69, 10, 16), (2, 11, 0, 3), (2, 0, 200, 33), (1, 30, 1, 2)]
    cutout_case(env, w, desc_rows)


@pytest.mark.parametrize("nchan", [1024, 4096, 8192])
def test_cutouts_tiled_bands(env, nchan):
    """Channel counts whose bands are whole 16-byte row segments: the batch
    kernel stages each band's raw rows in LDS where the rows of a bin plus
    the band's delay spread fit (and reads them directly where not: the
    high-DM trials of the D = 1 row)."""
    segs = [(0.0, 2.0, 40, 1), (80.0, 4.0, 20, 2), (160.0, 8.0, 12, 4)]
    w = synth.small(nchan=nchan, nsamp=9000, segments=segs, n_pulses=3, seed_offset=70 + nchan % 7,
                    widths=[1, 2, 4, 8, 16, 32, 64, 128])
    # (row, trial, t_peak, width), all inside their rows (n_out 8087, 3587, 1524)
    extra = [(0, 39, 3000, 128), (0, 0, 0, 64), (0, 20, 5, 9), (1, 19, 3400, 64), (2, 11, 1400, 100),
             (2, 0, 2, 40), (1, 7, 100, 1)]
    cutout_case(env, w, extra)


def test_cutouts_tiled_bands_high_dm(env):
    """Realistic sampling (4096 channels over 1000-1500 MHz, tsamp 49.152 us)
    at high DM, where a 64-channel band's delay spread plus a bin no longer
    fits the tile: the kernel stages such bands in 32-channel groups (D = 4
    row near DM 600: 199 samples of spread at the bottom of the band) or
    16-channel groups (D = 8 row near DM 1500: 247 samples), and the upper
    bands still in 64-channel groups."""
    segs = [(600.0, 1.0, 16, 4), (1480.0, 3.0, 12, 8)]
    w = synth.small(nchan=4096, nsamp=90000, segments=segs, tsamp=49.152e-6, n_pulses=2, seed_offset=91,
                    widths=[1, 2, 4, 8, 16, 32, 64])
    # (row, trial, t_peak, width) inside their rows (n_out 15288 and 2378)
    extra = [(0, 5, 3000, 64), (0, 15, 100, 8), (1, 6, 2000, 64), (1, 0, 10, 16), (1, 11, 2300, 8)]
    cutout_case(env, w, extra)


@pytest.mark.parametrize("case", ["multirow", "realistic_high_dm", "no_full_resolution_row"])
def test_cutouts_large_batch(env, case):
    """A batch of 300 candidates: the band sums come from a channel-major
    copy of the input: the copy the dedispersion's full-resolution row left
    staged, or, in a plan without such a row, one made for the cutouts.
    Bins of 16, 32 or 64 bytes wholly after the start are read as 16-byte
    chunks of each channel's window (the wide edge cases below: r D = 16, 32
    and 64), others one dword per lane and bin.  The oracle checks the
    search's candidates, the edge cases and every 9th random one."""
    if case == "no_full_resolution_row":
        segs = [(40.0, 2.0, 70, 2), (180.0, 4.0, 12, 4)]
        w = synth.small(nchan=192, nsamp=6000, segments=segs, n_pulses=3, seed_offset=61,
                        widths=[1, 2, 4, 8, 16, 32, 64])
        extra = [(0, 69, 10, 16), (1, 11, 0, 3), (1, 0, 200, 33), (0, 30, 1, 2)]
    elif case == "multirow":
        segs = [(0.0, 1.0, 40, 1), (40.0, 2.0, 70, 2), (180.0, 4.0, 12, 4)]
        w = synth.small(nchan=192, nsamp=6000, segments=segs, n_pulses=3, seed_offset=60,
                        widths=[1, 2, 4, 8, 16, 32, 64])
        extra = [(1, 69, 10, 16), (2, 11, 0, 3), (2, 0, 200, 33), (1, 30, 1, 2), (0, 0, 0, 1), (0, 39, 5546 - 64, 64)]
    else:
        segs = [(600.0, 1.0, 16, 4), (1480.0, 3.0, 12, 8), (0.0, 0.5, 24, 1)]
        w = synth.small(nchan=4096, nsamp=90000, segments=segs, tsamp=49.152e-6, n_pulses=2, seed_offset=91,
                        widths=[1, 2, 4, 8, 16, 32, 64])
        extra = [(0, 5, 3000, 64), (0, 15, 100, 8), (1, 6, 2000, 64), (1, 0, 10, 16), (1, 11, 2300, 8),
                 (2, 23, 0, 64), (2, 0, 1, 1), (0, 7, 4000, 32), (2, 10, 5000, 128), (2, 4, 6000, 256),
                 (2, 3, 8000, 512)]
    first = 12 + len(extra)  # at most: the search's top candidates + the edge cases
    cutout_case(env, w, extra, batch=300, check=list(range(first)) + list(range(first, 300, 9)))


def test_cutouts_on_a_split_row(env):
    """A wide band (256 channels over 270-1620 MHz) whose D = 1 row is split
    between the byte-quad and the 16-bit tiles: the cutouts take the row's
    delays and DM-time series like any other row's."""
    gsp, ctx, torch = env
    segs = [(0.0, 0.1, 200, 1), (20.0, 0.3, 40, 2)]
    w = synth.small(nchan=256, nsamp=40000, segments=segs, f_lo=270.0, f_hi=1620.0, n_pulses=2, seed_offset=35,
                    widths=[1, 2, 4, 8, 16, 32])
    desc = gsp.plan_shape(w.nsamp, w.freqs, w.tsamp, w.segments)
    assert ctx.row_shape(w.freqs, desc, 0)[4] == 3
    cutout_case(env, w, [(0, 0, 0, 1), (0, 199, 20000, 32), (1, 39, 100, 8), (0, 120, 5, 16)])


def test_cutouts_invalid_candidates_give_zero_images(env):
    gsp, ctx, torch = env
    w = synth.tiny()
    X = w.generate()
    fb = torch.from_numpy(X).cuda()
    desc = gsp.plan_shape(w.nsamp, w.freqs, w.tsamp, w.segments)
    dmt = ctx.dedisperse(fb, w.freqs, desc)
    bad = np.zeros(4, gsp.CAND_DTYPE)
    bad["seg"] = [1, 0, 0, -1]
    bad["dm_index"] = [0, 200, 3, 0]
    bad["t_peak"] = [10, 10, 14072, 10]
    bad["width"] = [4, 4, 1, 4]
    out = gsp.cutouts(ctx, fb, w.freqs, dmt, desc, bad).cpu().numpy()
    assert (out == 0).all()
