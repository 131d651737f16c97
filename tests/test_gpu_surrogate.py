"""GPU tests of the Fourier-mode MLP surrogate (BF16 MFMA training and inference) against
the FP64 oracle of oracle/mlp.py, called through the C ABI.

Tolerances: the GEMM operands are BF16 (unit roundoff 2^-9 with round to nearest), the
products accumulate in FP32.  Per layer the inputs and weights are rounded once each and
the activations once more, so a layer's output carries ~3 * 2^-9 ~ 6e-3 relative error
per element, averaged down over the dot products; the checks use 1e-2 (forward) and
3e-2 (gradients, one more rounding of dY and dZ) in relative L2 norm.  The oracle is run
on the BF16-rounded weights and inputs, so only the internal roundings remain.
"""

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _bf16_round(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _tiny(seed=5, width=128, n=8, modes=4, max_batch=256):
    import paper_1701_01608_amd as fks
    from oracle import mlp
    sur = fks.Surrogate(n=n, modes=modes, width=width, max_batch=max_batch)
    params = mlp.init_params([sur.n_in, width, width, sur.n_out], seed)
    rng = np.random.default_rng(seed + 100)
    params[1] = rng.normal(0, 0.1, params[1].shape)
    params[3] = rng.normal(0, 0.1, params[3].shape)
    params[5] = rng.normal(0, 0.1, params[5].shape)
    sur.set_params(params)
    return sur, params


def test_forward_matches_oracle():
    from oracle import mlp
    sur, params = _tiny()
    rng = np.random.default_rng(11)
    x = rng.standard_normal((256, sur.n_in))
    xd = torch.as_tensor(x, dtype=torch.float32).to(torch.bfloat16).cuda()
    y = sur.forward(xd).cpu().numpy()
    pr = [_bf16_round(p) if i % 2 == 0 else p for i, p in enumerate(params)]
    y_ref, _ = mlp.forward(pr, _bf16_round(x))
    err = _rel(y, y_ref)
    print(f"forward rel-L2 {err:.3e}")
    assert err <= 1e-2


def test_gradients_match_oracle():
    from oracle import mlp
    sur, params = _tiny(seed=6)
    rng = np.random.default_rng(12)
    x = rng.standard_normal((128, sur.n_in))
    t = rng.standard_normal((128, sur.n_out)) * 0.5
    xd = torch.as_tensor(x, dtype=torch.float32).to(torch.bfloat16).cuda()
    td = torch.as_tensor(t, dtype=torch.float32).cuda()
    loss = sur.train_step(xd, td, lr=0.0, update=False)
    torch.cuda.synchronize()
    g = sur.get_grads()
    pr = [_bf16_round(p) if i % 2 == 0 else p for i, p in enumerate(params)]
    loss_ref, g_ref = mlp.loss_and_grads(pr, _bf16_round(x), t)
    assert abs(loss.item() - loss_ref) <= 1e-2 * loss_ref
    names = ["W1", "b1", "W2", "b2", "W3", "b3"]
    for name, a, b in zip(names, g, g_ref):
        err = _rel(a, b)
        print(f"grad {name} rel-L2 {err:.3e}")
        assert err <= 3e-2, name
    # parameters untouched without update
    p_after = sur.get_params()
    for a, b in zip(p_after, params):
        assert np.array_equal(a, np.asarray(b, dtype=np.float32))


def test_large_tile_products_match_oracle():
    """The 256 x 256 tile products: output layer forward at batch 512 (2 x 128 tiles), its
    weight gradient (n^3 x width = 128 x 2 tiles) and the split-K input gradient through
    the transposed W3 (batch and width multiples of 256)."""
    from oracle import mlp
    sur, params = _tiny(seed=31, width=512, n=32, modes=8, max_batch=512)
    rng = np.random.default_rng(131)
    x = rng.standard_normal((512, sur.n_in))
    xd = torch.as_tensor(x, dtype=torch.float32).to(torch.bfloat16).cuda()
    y = sur.forward(xd).cpu().numpy()
    pr = [_bf16_round(p) if i % 2 == 0 else p for i, p in enumerate(params)]
    y_ref, _ = mlp.forward(pr, _bf16_round(x))
    err = _rel(y, y_ref)
    print(f"forward rel-L2 {err:.3e}")
    assert err <= 1e-2
    t = rng.standard_normal((256, sur.n_out)) * 0.5
    td = torch.as_tensor(t, dtype=torch.float32).cuda()
    loss = sur.train_step(xd[:256].contiguous(), td, lr=0.0, update=False)
    torch.cuda.synchronize()
    g = sur.get_grads()
    loss_ref, g_ref = mlp.loss_and_grads(pr, _bf16_round(x[:256]), t)
    assert abs(loss.item() - loss_ref) <= 1e-2 * loss_ref
    for name, a, b in zip(["W1", "b1", "W2", "b2", "W3", "b3"], g, g_ref):
        err = _rel(a, b)
        print(f"grad {name} rel-L2 {err:.3e}")
        assert err <= 3e-2, name


def test_adam_step_matches_oracle():
    from oracle import mlp
    sur, params = _tiny(seed=7)
    rng = np.random.default_rng(13)
    x = torch.as_tensor(rng.standard_normal((128, sur.n_in)), dtype=torch.float32).to(torch.bfloat16).cuda()
    t = torch.as_tensor(rng.standard_normal((128, sur.n_out)), dtype=torch.float32).cuda()
    p32 = [np.asarray(p, dtype=np.float32).astype(np.float64) for p in params]
    opt = mlp.Adam(p32, lr=1e-3)
    for _ in range(3):
        sur.train_step(x, t, lr=1e-3, update=True)
        torch.cuda.synchronize()
        g = [a.astype(np.float64) for a in sur.get_grads()]
        p32 = opt.step(p32, g)
        got = sur.get_params()
        for a, b in zip(got, p32):
            # FP32 update arithmetic against FP64: a few ulps of the parameter
            assert np.max(np.abs(a - b)) <= 1e-6 * max(1.0, np.max(np.abs(b)))


# (16, 12) has no pruned kernel and takes the full transform followed by the low modes
@pytest.mark.parametrize("n,modes,dtype,center", [(8, 4, "f32", False), (16, 8, "f64", False), (32, 8, "f32", False),
                                                   (16, 8, "f64", True), (32, 8, "f32", True), (24, 8, "f64", True),
                                                   (16, 4, "f32", True), (16, 12, "f32", True),
                                                   (16, 12, "f64", False)])
def test_features_match_oracle(n, modes, dtype, center):
    import paper_1701_01608_amd as fks
    from fks_inputs import perturbed_maxwellians
    from oracle import mlp
    L = 8.0 if n >= 16 else 4.0
    f = perturbed_maxwellians(n, L, 5, seed=21)
    plan = fks.Plan(n=n, L=L, R=L * 4 / (3 + 2 ** 0.5), a1=2, a2=2, dtype=dtype, max_cells=4)
    sur = fks.Surrogate(n=n, modes=modes, width=128, max_batch=128, center=center)
    fd = torch.as_tensor(f, dtype=plan.torch_dtype).cuda().contiguous()
    x, rho, mom = sur.features(plan, fd)
    x = x.float().cpu().numpy()
    rho = rho.cpu().numpy()
    mom = mom.cpu().numpy()
    for c in range(5):
        assert abs(mom[c, 0] - f[c].sum() * (2 * L / n) ** 3) <= 1e-6 * mom[c, 0]
        xr, rr = mlp.features(f[c], L, modes, center=center)
        # BF16 storage: 2^-8 relative to the magnitude (|x| <= 1), plus FP32 transform error
        assert np.max(np.abs(x[c] - xr)) <= 2.0 ** -8 * np.max(np.abs(xr)) + 1e-6
        assert abs(rho[c] - rr) <= 1e-6 * rr


def test_infer_indicator_and_fallback():
    import paper_1701_01608_amd as fks
    from fks_inputs import perturbed_maxwellians
    from oracle import mlp
    n, L, cells = 16, 8.0, 200
    f = perturbed_maxwellians(n, L, cells, seed=3)
    plan = fks.Plan(n=n, L=L, R=6.0, a1=4, a2=4, dtype="f32", max_cells=64)
    sur = fks.Surrogate(n=n, modes=8, width=128, max_batch=256)
    sur.set_params(mlp.init_params([sur.n_in, 128, 128, sur.n_out], 9))
    fd = torch.as_tensor(f, dtype=torch.float32).cuda().contiguous()
    q_spec = plan.collide(fd)
    r = torch.empty(cells, dtype=torch.float64, device="cuda")
    # no fallback: q = rho^2 y, indicator from the FP64 moments of q
    q_sur, nf = sur.infer(plan, fd, threshold=-1.0, indicator=r)
    assert nf == 0
    x, rho, _ = sur.features(plan, fd)
    xp = torch.zeros((256, sur.n_in), dtype=torch.bfloat16, device="cuda")
    xp[:cells] = x
    y = sur.forward(xp)[:cells]
    expect = (y * (rho * rho)[:, None]).reshape(cells, n, n, n)
    assert torch.allclose(q_sur, expect, rtol=1e-6, atol=0.0)
    qs = q_sur.double().cpu().numpy()
    rr = r.cpu().numpy()
    for c in range(0, cells, 37):
        assert abs(rr[c] - mlp.moment_indicator(qs[c], L)) <= 1e-9 + 1e-6 * rr[c]
    # threshold at the median: exactly the cells above it take the spectral Q
    thr = float(np.median(rr))
    q_h, nf = sur.infer(plan, fd, threshold=thr)
    above = rr > thr
    assert nf == int(above.sum())
    torch.cuda.synchronize()
    a = torch.as_tensor(above, device="cuda")
    assert torch.equal(q_h[a], q_spec[a])
    assert torch.equal(q_h[~a], q_sur[~a])
    # threshold 0 on an untrained net: every cell falls back, result = spectral Q
    q_all, nf = sur.infer(plan, fd, threshold=0.0)
    assert nf == cells
    assert torch.equal(q_all, q_spec)


@pytest.mark.parametrize("center", [False, True])
def test_ranked_fallback(center):
    # the absolute residual a = r ||Q_sur||_2 ranks the cells; per chunk the ceil(frac c)
    # largest fall back to the spectral Q (bit for bit), the others keep the surrogate's Q
    import paper_1701_01608_amd as fks
    from fks_inputs import perturbed_maxwellians
    from oracle import mlp
    n, L, cells, mb = 16, 8.0, 300, 128                       # three chunks: 128, 128, 44
    f = perturbed_maxwellians(n, L, cells, seed=4)
    plan = fks.Plan(n=n, L=L, R=6.0, a1=4, a2=4, dtype="f32", max_cells=64)
    sur = fks.Surrogate(n=n, modes=8, width=128, max_batch=mb, center=center)
    sur.set_params(mlp.init_params([sur.n_in, 128, 128, sur.n_out], 11))
    fd = torch.as_tensor(f, dtype=torch.float32).cuda().contiguous()
    q_spec = plan.collide(fd)
    r = torch.empty(cells, dtype=torch.float64, device="cuda")
    a = torch.empty(cells, dtype=torch.float64, device="cuda")
    q_sur, nf0 = sur.infer(plan, fd, threshold=-1.0, indicator=r)
    q_sur2, nf1 = sur.infer_ranked(plan, fd, 0.0, indicator=a)
    torch.cuda.synchronize()
    assert nf0 == 0 and nf1 == 0 and torch.equal(q_sur, q_sur2)
    expect = r * q_sur.double().flatten(1).norm(dim=1)
    assert torch.allclose(a, expect, rtol=1e-12, atol=0.0)
    frac = 0.3
    q_h, nf = sur.infer_ranked(plan, fd, frac)
    torch.cuda.synchronize()
    fell = np.zeros(cells, dtype=bool)
    an = a.cpu().numpy()
    for c0 in range(0, cells, mb):
        c = min(mb, cells - c0)
        k = int(np.ceil(frac * c))
        top = np.argsort(-an[c0:c0 + c])[:k]
        fell[c0 + top] = True
    assert nf == int(fell.sum())
    m = torch.as_tensor(fell, device="cuda")
    assert torch.equal(q_h[m], q_spec[m]) and torch.equal(q_h[~m], q_sur[~m])
    # all and nothing
    q_all, nf = sur.infer_ranked(plan, fd, 1.0)
    assert nf == cells and torch.equal(q_all, q_spec)
    with pytest.raises(fks.FKSError):
        sur.infer_ranked(plan, fd, 1.5)


def test_centred_targets_and_inference_match_oracle():
    """Centred surrogate: targets are Q(v + u) / (s rho^2) and predictions s rho^2 y(v - u),
    both by the exact spectral shift; checked against the oracle's shift of the GPU's own
    Q and network output, and the indicator against the oracle's on the result."""
    import paper_1701_01608_amd as fks
    from fks_inputs import perturbed_maxwellians
    from oracle import mlp
    n, L, cells, s = 16, 8.0, 130, 3e-3
    f = perturbed_maxwellians(n, L, cells, seed=5)
    plan = fks.Plan(n=n, L=L, R=6.0, a1=4, a2=4, dtype="f32", max_cells=64)
    sur = fks.Surrogate(n=n, modes=8, width=128, max_batch=256, out_scale=s, center=True)
    sur.set_params(mlp.init_params([sur.n_in, 128, 128, sur.n_out], 4))
    fd = torch.as_tensor(f, dtype=torch.float32).cuda().contiguous()
    x, rho, mom = sur.features(plan, fd)
    q = plan.collide(fd).reshape(cells, -1)
    t = sur.targets(plan, q, rho, mom).reshape(cells, n, n, n).double().cpu().numpy()
    qn = q.reshape(cells, n, n, n).double().cpu().numpy()
    rn = rho.double().cpu().numpy()
    for c in range(0, cells, 29):
        u = mlp.mean_velocity(f[c], L)
        ref = mlp.spectral_shift(qn[c], u, L) / (s * rn[c] ** 2)
        assert np.max(np.abs(t[c] - ref)) <= 1e-5 * np.max(np.abs(ref))
    r = torch.empty(cells, dtype=torch.float64, device="cuda")
    q_sur, nf = sur.infer(plan, fd, threshold=-1.0, indicator=r)
    assert nf == 0
    xp = torch.zeros((256, sur.n_in), dtype=torch.bfloat16, device="cuda")
    xp[:cells] = x
    y = sur.forward(xp)[:cells].reshape(cells, n, n, n).double().cpu().numpy()
    qs = q_sur.double().cpu().numpy()
    rr = r.cpu().numpy()
    for c in range(0, cells, 29):
        u = mlp.mean_velocity(f[c], L)
        ref = mlp.spectral_shift(s * rn[c] ** 2 * y[c], -u, L)
        assert np.max(np.abs(qs[c] - ref)) <= 1e-5 * np.max(np.abs(ref))
        assert abs(rr[c] - mlp.moment_indicator(qs[c], L)) <= 1e-9 + 1e-6 * rr[c]
    # fallback still selects exactly the cells above the threshold
    thr = float(np.median(rr))
    q_h, nf = sur.infer(plan, fd, threshold=thr)
    a = torch.as_tensor(rr > thr, device="cuda")
    assert nf == int(a.sum())
    assert torch.equal(q_h[a], plan.collide(fd)[a])


def test_full_size_inference_chunks():
    """n = 32 in the benchmark's launch configuration (chunks of 4096 cells, centred):
    threshold 0 sends every cell to the spectral path and must reproduce its Q exactly;
    without fallback, sampled cells equal the oracle's shift of the network output."""
    import paper_1701_01608_amd as fks
    from fks_inputs import perturbed_maxwellians_device
    from oracle import mlp
    n, L, cells, s = 32, 8.0, 8192 + 130, 3e-3
    plan = fks.Plan(n=n, L=L, R=6.0, a1=4, a2=4, dtype="f32", max_cells=4096)
    sur = fks.Surrogate(n=n, modes=8, width=1024, max_batch=4096, out_scale=s, center=True)
    sur.set_params(mlp.init_params([sur.n_in, 1024, 1024, sur.n_out], 2))
    f = perturbed_maxwellians_device(n, L, cells, seed=3)
    q_all, nf = sur.infer(plan, f, threshold=0.0)
    assert nf == cells
    q_spec = torch.empty_like(f)
    for c0 in range(0, cells, 4096):
        plan.collide(f[c0:c0 + 4096], q_spec[c0:c0 + 4096])
    assert torch.equal(q_all, q_spec)
    q_sur, nf = sur.infer(plan, f, threshold=-1.0)
    assert nf == 0
    idx = [0, 4095, 4096, cells - 1]
    x, rho, _ = sur.features(plan, f[idx].contiguous())
    xp = torch.zeros((128, sur.n_in), dtype=torch.bfloat16, device="cuda")
    xp[:len(idx)] = x
    y = sur.forward(xp)[:len(idx)].reshape(len(idx), n, n, n).double().cpu().numpy()
    fn = f[idx].double().cpu().numpy()
    rn = rho.double().cpu().numpy()
    qs = q_sur[idx].double().cpu().numpy()
    for j in range(len(idx)):
        ref = mlp.spectral_shift(s * rn[j] ** 2 * y[j], -mlp.mean_velocity(fn[j], L), L)
        assert np.max(np.abs(qs[j] - ref)) <= 1e-5 * np.max(np.abs(ref))


def test_training_learns_operator():
    """Train online (fresh perturbed Maxwellians every 8192 samples, labelled by the FP32
    spectral path, n = 16), then check the held-out error against the oracle's Q on
    sampled cells, and that the moment indicator ranks cells by their true error."""
    import paper_1701_01608_amd as fks
    from fks_inputs import perturbed_maxwellians, perturbed_maxwellians_device
    from oracle import mlp
    from oracle.collide import collide_fast
    from oracle.tables import make_plan
    n, L, R = 16, 8.0, 6.0
    plan = fks.Plan(n=n, L=L, R=R, a1=4, a2=4, dtype="f32", max_cells=4096)
    width, batch, chunk, steps = 512, 512, 8192, 3000
    sur = fks.Surrogate(n=n, modes=8, width=width, max_batch=1024, out_scale=3e-3, center=True)
    sur.set_params(mlp.init_params([sur.n_in, width, width, sur.n_out], 1))
    losses, s, rnd = [], 0, 0
    while s < steps:
        f = perturbed_maxwellians_device(n, L, chunk, seed=1000 + rnd)
        x, rho, mom = sur.features(plan, f)
        t = sur.targets(plan, plan.collide(f).reshape(chunk, -1), rho, mom)
        rnd += 1
        for j in range(0, chunk, batch):
            lr = 1e-3 * 0.5 * (1 + np.cos(np.pi * s / steps))
            loss = sur.train_step(x[j:j + batch], t[j:j + batch], lr=lr)
            if s % 250 == 0 or s == steps - 1:
                losses.append(loss.item())
            s += 1
            if s >= steps:
                break
    print("losses", ["%.3e" % v for v in losses])
    assert losses[-1] < 0.2 * losses[0]
    # held-out cells (seed 2): surrogate vs the spectral Q, and vs the oracle on a sample
    n_val = 512
    f_val_np = perturbed_maxwellians(n, L, n_val, seed=2)
    f_val = torch.as_tensor(f_val_np, dtype=torch.float32).cuda()
    r = torch.empty(n_val, dtype=torch.float64, device="cuda")
    q_sur, _ = sur.infer(plan, f_val, threshold=-1.0, indicator=r)
    q_spec = plan.collide(f_val)
    d = (q_sur - q_spec).double().flatten(1)
    err = (d.norm(dim=1) / q_spec.double().flatten(1).norm(dim=1)).cpu().numpy()
    glob = float(d.norm() / q_spec.double().norm())
    print("surrogate rel-L2 %.3e; per cell median %.3e max %.3e" % (glob, np.median(err), err.max()))
    oplan = make_plan(n, L, R, a1=4, a2=4)
    for c in range(0, n_val, 170):
        q_ref = collide_fast(f_val_np[c], oplan)
        e_ref = np.linalg.norm(q_sur[c].double().cpu().numpy() - q_ref) / np.linalg.norm(q_ref)
        assert abs(e_ref - err[c]) <= 1e-4 + 1e-3 * err[c]  # spectral FP32 Q is within 1e-5 of the oracle
    assert glob < 0.5 and np.median(err) < 0.5
    # the indicator ranks cells by true error (Spearman rank correlation)
    rr = r.cpu().numpy()
    rank_r = np.argsort(np.argsort(rr))
    rank_e = np.argsort(np.argsort(err))
    corr = np.corrcoef(rank_r, rank_e)[0, 1]
    print("indicator/error rank correlation %.3f" % corr)
    assert corr > 0.3
    # the hybrid: lowering the threshold moves cells to the spectral path; the fallback
    # count never drops, the error against the spectral Q never rises, and threshold 0
    # reproduces the spectral Q exactly
    q2 = q_spec.double().pow(2).sum()
    prev_nf, prev_err = -1, np.inf
    for thr in (np.inf, float(np.quantile(rr, 0.75)), float(np.median(rr)), float(np.quantile(rr, 0.25)), 0.0):
        q_h, nf = sur.infer(plan, f_val, threshold=thr)
        e = float(((q_h - q_spec).double().pow(2).sum() / q2).sqrt())
        print(f"threshold {thr:.3e}: fallback {nf}/{n_val}, rel-L2 {e:.3e}")
        assert nf >= prev_nf and e <= prev_err * (1 + 1e-9) + 1e-12
        prev_nf, prev_err = nf, e
    assert nf == n_val and torch.equal(q_h, q_spec)


def test_trained_surrogate_gain_over_spectral_path():
    """What the learned part gains: on 4096 held-out cells at n = 32 the trained network's
    Q is far closer to the spectral Q than the untrained network's, and its inference runs
    several times faster than the spectral evaluation of the same cells (the benchmark's
    longer training reaches 5 % at about 12x)."""
    import time
    import paper_1701_01608_amd as fks
    from fks_inputs import mlp_init, perturbed_maxwellians_device
    n, L, R, cells = 32, 8.0, 6.0, 4096
    plan = fks.Plan(n, L, R, a1=4, a2=4, C=0.25, dtype="f32", max_cells=cells)
    sur = fks.Surrogate(n=n, modes=8, width=1024, max_batch=cells, out_scale=3e-3, center=True)
    sur.set_params(mlp_init([sur.n_in, 1024, 1024, sur.n_out], 1))
    f_val = perturbed_maxwellians_device(n, L, cells, seed=2)
    q_spec = plan.collide(f_val)

    def rel_err():
        q_sur, _ = sur.infer(plan, f_val, threshold=-1.0)
        return float((q_sur - q_spec).double().norm() / q_spec.double().norm())

    e0 = rel_err()
    pairs, batch, steps = 8192, 1024, 1500
    f_tr = perturbed_maxwellians_device(n, L, pairs, seed=1000)
    x, rho, mom = sur.features(plan, f_tr)
    t = sur.targets(plan, plan.collide(f_tr).reshape(pairs, -1), rho, mom)
    for s in range(steps):
        j = (s * batch) % pairs
        sur.train_step(x[j:j + batch], t[j:j + batch], lr=1e-3 * 0.5 * (1 + np.cos(np.pi * s / steps)))
    torch.cuda.synchronize()
    e1 = rel_err()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        best = np.inf
        for _ in range(3):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        return best

    q_out = torch.empty_like(f_val)
    t_sur = timed(lambda: sur.infer(plan, f_val, q=q_out, threshold=-1.0))
    t_spec = timed(lambda: plan.collide(f_val, q_out))
    print(f"rel-L2 untrained {e0:.3e} trained {e1:.3e}; surrogate {t_sur * 1e3:.3f} ms, "
          f"spectral {t_spec * 1e3:.3f} ms ({t_spec / t_sur:.1f}x)")
    assert e1 < 0.5 and e1 < 0.5 * e0
    assert t_spec > 3.0 * t_sur
    # at an equal fallback share (half the cells), ranking the cells by the absolute
    # residual r ||Q_sur|| leaves a smaller batch error than a threshold on the relative
    # residual r: the batch rel-L2 is carried by the cells with the largest Q
    r = torch.empty(cells, dtype=torch.float64, device="cuda")
    sur.infer(plan, f_val, threshold=-1.0, indicator=r)
    thr = float(torch.quantile(r, 0.5))
    q_rel, n_rel = sur.infer(plan, f_val, threshold=thr)
    q_abs, n_abs = sur.infer_ranked(plan, f_val, n_rel / cells)
    e_rel = float((q_rel - q_spec).double().norm() / q_spec.double().norm())
    e_abs = float((q_abs - q_spec).double().norm() / q_spec.double().norm())
    print(f"fallback {n_rel} cells: relative-threshold {e_rel:.3e}, ranked absolute {e_abs:.3e}")
    assert abs(n_abs - n_rel) <= 1 and e_abs < e_rel < e1
