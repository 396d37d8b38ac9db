"""GPU surrogate network against the FP64 oracle (oracle/mlp.py).

The GPU keeps W2..W5 and the hidden activations in bf16 (fp32 accumulation,
fp32 first layer and biases).  The oracle is fed the same bf16-rounded
weights; an emulation that also rounds the activations pins the kernels
tightly, the plain FP64 forward within 1e-2 on probabilities.  Gradients are
compared per layer by cosine (>= 0.999) and relative L2 (<= 2e-2).
"""
import struct

import numpy as np
import pytest

from oracle import mlp

pytestmark = pytest.mark.gpu

P = 200451
SIZES = (8, 256, 256, 256, 256, 3)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.fixture()
def ctx(torch):
    from paper_2409_00165_amd import fos
    c = fos.Context(0)
    yield c.handle
    c.close()


def _flat(params):
    out = []
    for W, b in params:
        out.append(np.asarray(W, np.float64).reshape(-1))
        out.append(np.asarray(b, np.float64).reshape(-1))
    v = np.concatenate(out)
    assert v.size == P
    return v


def _unflat(v):
    params, o = [], 0
    for k, n in zip(SIZES[:-1], SIZES[1:]):
        W = v[o:o + k * n].reshape(k, n); o += k * n
        b = v[o:o + n]; o += n
        params.append((W, b))
    return params


def _blob(members, mean, std, lo, hi):
    stats = np.concatenate([mean, 1.0 / std, lo, hi]).astype(np.float32)
    hdr = b"FOSSUR01" + struct.pack("<6I", 4, 8, 256, P, 1, 0)
    w = np.stack([_flat(p) for p in members]).astype(np.float32)
    z = np.zeros_like(w)
    return hdr + stats.tobytes() + w.tobytes() + z.tobytes() + z.tobytes()


def _model(seed=0):
    members = []
    rng = np.random.default_rng(seed + 100)
    for m in range(4):
        p = mlp.init(seed * 10 + m)
        p = [(W, rng.normal(0, 0.1, b.shape)) for W, b in p]
        members.append(p)
    mean = np.array([0.5, -1.0, 0.4, 1.5, 1.8, -2.0, 0.75, 0.0])
    std = np.array([1.7, 1.3, 0.25, 0.12, 0.7, 0.9, 0.14, 1.0])
    lo = mean - 3 * std
    hi = mean + 3 * std
    lo[7] = hi[7] = 0.0
    return members, mean, std, lo, hi


def _as_gpu_weights(params):
    """fp32 W1/biases, bf16 W2..W5 -- what the kernels multiply with."""
    out = []
    for i, (W, b) in enumerate(params):
        W32 = np.asarray(W, np.float32).astype(np.float64)
        out.append((W32 if i == 0 else mlp.to_bf16(W), np.asarray(b, np.float32).astype(np.float64)))
    return out


def _emulated_forward(params, xs):
    """Forward with the activations rounded to bf16 as the GPU stores them."""
    h = xs
    for i, (W, b) in enumerate(params[:-1]):
        h = mlp.to_bf16(mlp.gelu(h @ W + b))
    W, b = params[-1]
    return mlp.softmax(h @ W + b)


def _features(n, seed=1, mean=None, std=None):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(n, 8)) * std + mean
    x[:, 7] = 0.0
    return x.astype(np.float32)


def test_forward_members_match_oracle(ctx, torch):
    from paper_2409_00165_amd import fos
    members, mean, std, lo, hi = _model(0)
    fos.fos_sur_load(ctx, _blob(members, mean, std, lo, hi))
    n = 1000
    x = _features(n, 1, mean, std)
    dx = torch.from_numpy(x).cuda()
    rat = torch.zeros(n * 3, device="cuda")
    spread = torch.zeros(n, device="cuda")
    ind = torch.zeros(n, dtype=torch.uint8, device="cuda")
    mem = torch.zeros(4 * n * 3, device="cuda")
    fos.fos_sur_predict(ctx, dx, rat=rat, spread=spread, in_domain=ind, members=mem)
    torch.cuda.synchronize()
    mem = mem.cpu().numpy().reshape(4, n, 3).astype(np.float64)
    xs = (x.astype(np.float64) - mean) / std
    xs = xs.astype(np.float32).astype(np.float64)
    worst_em, worst_fp = 0.0, 0.0
    for m in range(4):
        gw = _as_gpu_weights(members[m])
        em = _emulated_forward(gw, xs)
        fp, _ = mlp.forward(gw, xs)
        worst_em = max(worst_em, np.abs(mem[m] - em).max())
        worst_fp = max(worst_fp, np.abs(mem[m] - fp).max())
    print("forward max |dp|: vs bf16-emulating oracle", worst_em, "vs fp64 oracle", worst_fp, flush=True)
    assert worst_em < 5e-3     # one-ulp bf16 flips of hidden activations (fp32 vs fp64 sums)
    assert worst_fp < 1e-2
    r = rat.cpu().numpy().reshape(n, 3)
    assert np.allclose(r, mem.mean(0), atol=1e-6)
    assert np.allclose(r.sum(1), 1.0, atol=1e-5)
    assert np.allclose(spread.cpu().numpy(), (mem.max(0) - mem.min(0)).max(1), atol=1e-6)


def test_prediction_spans_many_tiles_row_independently(ctx, torch):
    """200,003 rows (1,563 workgroups of 128, ragged last tile): rows predicted
    in a small call are bit-identical inside the large call (head and tail),
    and sampled rows match the bf16-emulating oracle."""
    from paper_2409_00165_amd import fos
    members, mean, std, lo, hi = _model(5)
    fos.fos_sur_load(ctx, _blob(members, mean, std, lo, hi))
    n = 200_003
    x = _features(n, 11, mean, std)
    dx = torch.from_numpy(x).cuda()

    def run(xx):
        m = xx.shape[0]
        out = (torch.zeros(m * 3, device="cuda"), torch.zeros(m, device="cuda"),
               torch.zeros(m, dtype=torch.uint8, device="cuda"), torch.zeros(4 * m * 3, device="cuda"))
        fos.fos_sur_predict(ctx, xx.reshape(-1), rat=out[0], spread=out[1], in_domain=out[2], members=out[3])
        return out

    big = run(dx)
    head = run(dx[:1000].contiguous())
    tail = run(dx[-77:].contiguous())
    torch.cuda.synchronize()
    bm = big[3].view(4, n, 3)
    assert torch.equal(big[0].view(n, 3)[:1000], head[0].view(1000, 3))
    assert torch.equal(big[1][:1000], head[1]) and torch.equal(big[2][:1000], head[2])
    assert torch.equal(bm[:, :1000], head[3].view(4, 1000, 3))
    assert torch.equal(big[0].view(n, 3)[-77:], tail[0].view(77, 3))
    assert torch.equal(bm[:, -77:], tail[3].view(4, 77, 3))
    rows = np.random.default_rng(12).choice(n, size=300, replace=False)
    xs = ((x[rows].astype(np.float64) - mean) / std).astype(np.float32).astype(np.float64)
    got = bm[:, torch.from_numpy(rows).cuda()].cpu().numpy().astype(np.float64)
    worst = 0.0
    for m in range(4):
        worst = max(worst, np.abs(got[m] - _emulated_forward(_as_gpu_weights(members[m]), xs)).max())
    print("sampled rows of the 200,003-row call vs bf16-emulating oracle:", worst, flush=True)
    assert worst < 5e-3


def test_prediction_at_full_sweep_size(ctx, torch):
    """2e8 rows in one launch, the size of the paint sweep (10^6 designs x
    200 wavelengths; 1,562,500 workgroups): the first and last 64 rows and 300
    at random against the bf16-emulating oracle (ensemble mean and spread), and
    the domain flag against the training box checked on the host."""
    from paper_2409_00165_amd import fos
    members, mean, std, lo, hi = _model(7)
    fos.fos_sur_load(ctx, _blob(members, mean, std, lo, hi))
    n = 200_000_000
    gen = torch.Generator(device="cuda")
    gen.manual_seed(2024)
    x = torch.randn(n, 8, device="cuda", generator=gen)
    x.mul_(torch.from_numpy(std.astype(np.float32)).cuda()).add_(torch.from_numpy(mean.astype(np.float32)).cuda())
    x[:, 7] = 0.0
    rat = torch.zeros(n * 3, device="cuda")
    spread = torch.zeros(n, device="cuda")
    ind = torch.zeros(n, dtype=torch.uint8, device="cuda")
    fos.fos_sur_predict(ctx, x.view(-1), rat=rat, spread=spread, in_domain=ind)
    torch.cuda.synchronize()
    rows = np.concatenate([np.arange(64), np.arange(n - 64, n),
                           np.random.default_rng(13).choice(n, size=300, replace=False)])
    ri = torch.from_numpy(rows).cuda()
    xr = x[ri].cpu().numpy()
    got_rat = rat.view(n, 3)[ri].cpu().numpy().astype(np.float64)
    got_spread = spread[ri].cpu().numpy().astype(np.float64)
    got_in = ind[ri].cpu().numpy()
    del x, rat, spread, ind
    torch.cuda.empty_cache()
    xs = ((xr.astype(np.float64) - mean) / std).astype(np.float32).astype(np.float64)
    em = np.stack([_emulated_forward(_as_gpu_weights(m), xs) for m in members])
    d_rat = np.abs(got_rat - em.mean(0)).max()
    d_spread = np.abs(got_spread - (em.max(0) - em.min(0)).max(1)).max()
    print("2e8-row call, sampled rows vs bf16-emulating oracle: mean", d_rat, "spread", d_spread, flush=True)
    assert d_rat < 5e-3 and d_spread < 1e-2
    box = np.all((xr >= lo.astype(np.float32)) & (xr <= hi.astype(np.float32)), axis=1)
    assert np.array_equal(got_in.astype(bool), box)
    assert 0 < box.sum() < len(rows)


def test_gate_domain_and_eligibility(ctx, torch):
    from paper_2409_00165_amd import fos
    members, mean, std, lo, hi = _model(1)
    fos.fos_sur_load(ctx, _blob(members, mean, std, lo, hi))
    x = np.tile(mean.astype(np.float32), (6, 1))
    x[1, 0] = hi[0] + 0.01          # above the box
    x[2, 3] = lo[3] - 0.01          # below the box
    x[3, 7] = 1.0                   # not layer 0
    elig = np.array([1, 1, 1, 1, 0, 1], np.uint8)
    ind = torch.zeros(6, dtype=torch.uint8, device="cuda")
    fos.fos_sur_predict(ctx, torch.from_numpy(x).cuda(), eligible=torch.from_numpy(elig).cuda(), in_domain=ind)
    torch.cuda.synchronize()
    assert list(ind.cpu().numpy()) == [1, 0, 0, 0, 0, 1]


def _check_grads(g_gpu, g_ref, label):
    for li in range(5):
        for j, name in ((0, "W"), (1, "b")):
            a = g_gpu[li][j].ravel()
            b = g_ref[li][j].ravel()
            cos = float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-300))
            rel = float(np.linalg.norm(a - b) / (np.linalg.norm(b) + 1e-300))
            assert cos >= 0.999 and rel <= 2e-2, (label, li, name, cos, rel)


@pytest.mark.parametrize("n", [512, 2048, 8192, 2112])
def test_gradients_match_oracle_backprop(ctx, torch, n):
    """Gradients of the mean loss over n rows: the weight gradients reduce
    over the rows in K ranges (2 at 512 rows, 8 at 2048, 16 at 8192, and 2
    ranges of 33 k-steps at 2112 rows), each checked against backprop of the
    FP64 oracle."""
    from paper_2409_00165_amd import fos
    members, mean, std, lo, hi = _model(2)
    fos.fos_sur_load(ctx, _blob(members, mean, std, lo, hi))
    x = _features(n, 3, mean, std)
    y = np.random.default_rng(4).dirichlet(np.ones(3), size=n).astype(np.float32)
    grads = torch.zeros(4 * P, device="cuda")
    loss = torch.zeros(4, device="cuda")
    fos.fos_sur_grad(ctx, torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda(), grads, loss)
    torch.cuda.synchronize()
    g = grads.cpu().numpy().reshape(4, P).astype(np.float64)
    lg = loss.cpu().numpy()
    xs = ((x.astype(np.float64) - mean) / std).astype(np.float32).astype(np.float64)
    for m in range(4):
        gw = _as_gpu_weights(members[m])
        p, cache = mlp.forward(gw, xs)
        ref = mlp.backward(gw, cache, p, y.astype(np.float64))
        _check_grads(_unflat(g[m]), ref, f"member {m}")
        assert abs(lg[m] - mlp.loss(p, y)) < 2e-3 * max(1.0, mlp.loss(p, y))


def test_adam_step_matches_oracle(ctx, torch):
    from paper_2409_00165_amd import fos
    members, mean, std, lo, hi = _model(3)
    fos.fos_sur_load(ctx, _blob(members, mean, std, lo, hi))
    n = 256
    x = _features(n, 5, mean, std)
    y = np.random.default_rng(6).dirichlet(np.ones(3), size=n).astype(np.float32)
    dx, dy = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    grads = torch.zeros(4 * P, device="cuda")
    fos.fos_sur_grad(ctx, dx, dy, grads)
    torch.cuda.synchronize()
    g = grads.cpu().numpy().reshape(4, P).astype(np.float64)
    lr = 1e-3
    fos.fos_sur_train(ctx, dx, dy, epochs=1, batch=n, lr=lr, lr_min=lr, seed=9, resume=True)
    torch.cuda.synchronize()
    _, new, step = fos.parse_sur_blob(fos.fos_sur_save(ctx))
    assert step == 1
    for m in range(4):
        p0 = [(np.asarray(W, np.float32).astype(np.float64), np.asarray(b, np.float32).astype(np.float64))
              for W, b in members[m]]
        opt = mlp.Adam(p0, lr=lr)
        ref = _flat(opt.step(p0, _unflat(g[m])))
        d = np.abs(new[m].astype(np.float64) - ref)
        # the shuffled batch sums the same rows in another order: only weights
        # whose gradient is ~0 may step the other way
        assert (d > 1e-6).mean() < 2e-3, (m, (d > 1e-6).mean())


def test_save_load_round_trip_is_bit_exact(ctx, torch):
    from paper_2409_00165_amd import fos
    members, mean, std, lo, hi = _model(4)
    fos.fos_sur_load(ctx, _blob(members, mean, std, lo, hi))
    blob = fos.fos_sur_save(ctx)
    x = torch.from_numpy(_features(300, 7, mean, std)).cuda()
    a = torch.zeros(900, device="cuda")
    fos.fos_sur_predict(ctx, x, rat=a)
    c2 = fos.Context(0)
    fos.fos_sur_load(c2.handle, blob)
    b = torch.zeros(900, device="cuda")
    fos.fos_sur_predict(c2.handle, x, rat=b)
    torch.cuda.synchronize()
    c2.close()
    assert torch.equal(a, b)


def test_training_reduces_the_loss(ctx, torch):
    from paper_2409_00165_amd import fos
    rng = np.random.default_rng(8)
    n = 32768
    x = rng.normal(size=(n, 8)).astype(np.float32)
    x[:, 7] = 0
    logits = np.stack([1.5 * np.tanh(x[:, 0]), x[:, 1] * x[:, 2] * 0.5, -0.7 * x[:, 3] + 0.3 * x[:, 4]], 1)
    y = mlp.softmax(logits).astype(np.float32)
    hist = torch.zeros(6 * 4, device="cuda")
    fos.fos_sur_train(ctx, torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda(), epochs=6, batch=1024,
                      lr=2e-3, lr_min=1e-4, seed=3, loss_history=hist)
    torch.cuda.synchronize()
    h = hist.cpu().numpy().reshape(6, 4)
    ent = mlp.loss(y.astype(np.float64), y.astype(np.float64))
    print("loss history - entropy:\n", h - ent, flush=True)
    assert (h[-1] < h[0]).all()
    assert (h[-1] - ent < 0.1 * (h[0] - ent)).all()
    rat = torch.zeros(n * 3, device="cuda")
    fos.fos_sur_predict(ctx, torch.from_numpy(x).cuda(), rat=rat)
    torch.cuda.synchronize()
    err = np.abs(rat.cpu().numpy().reshape(n, 3) - y).max(1)
    print("fit: mean |dp|", err.mean(), "p99", np.quantile(err, 0.99), flush=True)
    assert err.mean() < 0.02
