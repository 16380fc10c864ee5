"""The learned CG start on the GPU: descriptors, targets, gradients against
the FP64 reference, BF16 inference, start parity, residual-judged fallback,
and the effect of a (briefly) trained network."""

import math
import sys

import numpy as np
import pytest

from paper_1202_0098_amd import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1202_0098_amd as ma
    ctx = ma.Context(0)
    s = synth.config_diamond4096()
    ctx.build_tb(s)
    ctx.mlp_init(seed=3)
    yield torch, ma, ctx, s
    ctx.close()


def _nearest(s, A, k):
    d = s.pos - s.pos[A]
    d -= s.box * np.round(d / s.box)
    d2 = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2]
    order = np.lexsort((np.arange(s.n_atoms), d2))[:k]
    return order, d[order], np.sqrt(d2[order])


def test_descriptors(env):
    torch, ma, ctx, s = env
    sh = ctx.mlp_shape()
    assert sh["n_in"] == 192 + 4 and sh["n_out"] == 48 and sh["n_hidden"] == 256
    cols = np.array([0, 5, 4095 * 4 + 3, 9001], np.int32)
    feat = torch.zeros(len(cols) * sh["n_in"], dtype=torch.float32, device="cuda")
    ctx.column_features(cols, feat)
    f = feat.cpu().numpy().reshape(len(cols), -1)
    for c, j in enumerate(cols):
        A, r = divmod(int(j), 4)
        idx, dv, dist = _nearest(s, A, 49)
        exp = np.zeros(sh["n_in"])
        for k in range(1, 49):
            exp[4 * (k - 1)] = dist[k] / 5.0
            exp[4 * (k - 1) + 1:4 * k] = dv[k] / dist[k]
        exp[192 + r] = 1.0
        assert np.abs(f[c] - exp).max() < 1e-6


def test_sj_targets_match_oracle(env):
    torch, ma, ctx, s = env
    import oracle
    cols = np.array([3, 777, 12345], np.int32)
    sj = torch.zeros(len(cols) * 48, dtype=torch.float32, device="cuda")
    ctx.solve_columns(cols, 1, 0, mu=0.0, kT=s.kT, sj_near=sj)
    got = sj.cpu().numpy().reshape(len(cols), 48)
    raw = oracle.solve_raw(s, cols, p=1, q=0, want_sj=True)
    for c, j in enumerate(cols):
        A, r = divmod(int(j), 4)
        reg = oracle.region_of(s.pos, s.box, A, "nearest", 0, 120)
        idx, _, _ = _nearest(s, A, 12)
        exp = np.concatenate([raw["sj"][c, int(np.searchsorted(reg, b)) * 4:
                                        int(np.searchsorted(reg, b)) * 4 + 4] for b in idx])
        assert np.abs(got[c] - exp).max() < 1e-6
        assert abs(got[c, r] - 1.0) < 0.2       # S ~ I: s_j is close to e_j


def test_gradient_matches_fp64_reference(env):
    torch, ma, ctx, s = env
    from oracle import mlp
    sh = ctx.mlp_shape()
    shape = (sh["n_in"], sh["n_hidden"], sh["n_out"])
    rng = np.random.default_rng(11)
    n = 96
    X = rng.normal(size=(n, sh["n_in"])).astype(np.float32)
    T = (rng.normal(size=(n, sh["n_out"])) * 0.1).astype(np.float32)
    params = ctx.mlp_get_params()
    Xd = torch.from_numpy(X).cuda()
    Td = torch.from_numpy(T).cuda()
    loss, g = ctx.mlp_loss_grad(Xd, Td, n)
    loss_o, g_o = mlp.loss_grad(params.astype(np.float64), X.astype(np.float64),
                                T.astype(np.float64), shape)
    _say(f"loss gpu {loss:.8e} ref {loss_o:.8e}; grad rel err "
         f"{np.linalg.norm(g - g_o) / np.linalg.norm(g_o):.2e}")
    assert abs(loss - loss_o) < 1e-5 * loss_o
    assert np.linalg.norm(g - g_o) <= 1e-4 * np.linalg.norm(g_o)
    # with a row gather
    idx = np.array(rng.permutation(n)[:40], np.int32)
    loss2, g2 = ctx.mlp_loss_grad(Xd, Td, 40, idx=torch.from_numpy(idx).cuda())
    loss2_o, g2_o = mlp.loss_grad(params.astype(np.float64), X[idx].astype(np.float64),
                                  T[idx].astype(np.float64), shape)
    assert np.linalg.norm(g2 - g2_o) <= 1e-4 * np.linalg.norm(g2_o)


def test_adam_step_matches_reference(env):
    torch, ma, ctx, s = env
    from oracle import mlp
    sh = ctx.mlp_shape()
    shape = (sh["n_in"], sh["n_hidden"], sh["n_out"])
    rng = np.random.default_rng(12)
    n = 64
    X = rng.normal(size=(n, sh["n_in"])).astype(np.float32)
    T = (rng.normal(size=(n, sh["n_out"])) * 0.1).astype(np.float32)
    ctx.mlp_init(seed=5)
    p0 = ctx.mlp_get_params().astype(np.float64)
    ctx.mlp_train_step(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda(), n, 1e-3)
    p1 = ctx.mlp_get_params().astype(np.float64)
    _, g = mlp.loss_grad(p0, X.astype(np.float64), T.astype(np.float64), shape)
    p1_o, _, _ = mlp.adam_step(p0, g, np.zeros_like(p0), np.zeros_like(p0), 1, 1e-3)
    # the first Adam step is lr * sign(g) except where |g| ~ eps
    big = np.abs(g) > 1e-5
    assert np.abs(p1 - p1_o)[big].max() < 1e-6
    ctx.mlp_init(seed=3)


def test_bf16_inference_close_to_fp32(env):
    torch, ma, ctx, s = env
    sh = ctx.mlp_shape()
    cols = np.arange(0, s.M, 37, dtype=np.int32)
    n = len(cols)
    feat = torch.zeros(n * sh["n_in"], dtype=torch.float32, device="cuda")
    ctx.column_features(cols, feat)
    y16 = torch.zeros(n * sh["n_out"], dtype=torch.float32, device="cuda")
    y32 = torch.zeros_like(y16)
    ctx.mlp_forward(feat, n, y16, bf16=True)
    ctx.mlp_forward(feat, n, y32, bf16=False)
    a, b = y16.cpu().numpy(), y32.cpu().numpy()
    rel = np.linalg.norm(a - b) / np.linalg.norm(b)
    _say(f"bf16 vs fp32 inference relative difference {rel:.2e}")
    assert rel < 3e-2


def test_inference_matches_fp64_reference(env):
    """Both inference paths against the FP64 reference network, element by
    element.  BF16 rounds the weights and the layer inputs to 8 significant
    bits (relative 2^-9 each); through three layers the error of output k is
    bounded by a small multiple of that times the magnitude network
    |x||W1| + |b1| -> |silu| -> ... evaluated with absolute values: 0.02 of
    it is used.  The FP32 path is held to 1e-5 of the same magnitude."""
    torch, ma, ctx, s = env
    from oracle import mlp
    sh = ctx.mlp_shape()
    shape = (sh["n_in"], sh["n_hidden"], sh["n_out"])
    cols = np.arange(0, s.M, 53, dtype=np.int32)
    n = len(cols)
    feat = torch.zeros(n * sh["n_in"], dtype=torch.float32, device="cuda")
    ctx.column_features(cols, feat)
    y16 = torch.zeros(n * sh["n_out"], dtype=torch.float32, device="cuda")
    y32 = torch.zeros_like(y16)
    ctx.mlp_forward(feat, n, y16, bf16=True)
    ctx.mlp_forward(feat, n, y32, bf16=False)
    x = feat.cpu().numpy().reshape(n, -1).astype(np.float64)
    params = ctx.mlp_get_params().astype(np.float64)
    ref = mlp.forward(params, x, shape)
    ref = ref[0] if isinstance(ref, tuple) else ref
    W1, b1, W2, b2, W3, b3 = mlp.unpack(params, *shape)
    m1 = np.abs(x) @ np.abs(W1) + np.abs(b1)
    m2 = m1 @ np.abs(W2) + np.abs(b2)          # |silu(z)| <= |z|
    scale = m2 @ np.abs(W3) + np.abs(b3)
    a16 = y16.cpu().numpy().reshape(n, -1)
    a32 = y32.cpu().numpy().reshape(n, -1)
    r16 = float(np.max(np.abs(a16 - ref) / scale))
    r32 = float(np.max(np.abs(a32 - ref) / scale))
    _say(f"inference vs FP64 reference: bf16 {r16:.2e}, fp32 {r32:.2e} of the magnitude bound")
    assert r16 <= 0.02
    assert r32 <= 1e-5


def test_learned_start_gives_same_result_and_fallback(env):
    torch, ma, ctx, s = env
    import oracle
    cols = np.sort(np.random.default_rng(3).choice(s.M, 160, replace=False)).astype(np.int32)
    o = s.n_orb
    out = {}
    for start in ["zero", "learned"]:
        rho = torch.zeros(s.nblk * o * o, dtype=torch.float64, device="cuda")
        st = torch.zeros(len(cols) * ma.STATS, dtype=torch.int32, device="cuda")
        r = ctx.solve_columns(cols, s.p, s.q, mu=0.95, kT=s.kT, rho=rho, col_stats=st,
                              opts=ma.default_opts(start=start))
        out[start] = (r, rho.cpu().numpy(), st.cpu().numpy().reshape(-1, ma.STATS))
    ref = oracle.solve(s, cols=cols, mu=0.95)
    rho_o = oracle.scatter_slots(s, cols, ref["rho"]).ravel()
    for start in out:
        assert np.abs(out[start][1] - rho_o).max() < 1e-10
    assert np.all(out["zero"][2][:, 4] == 0)
    assert np.all(out["learned"][2][:, 4] >= 1)
    # force rejection of every predicted start with a huge output bias
    p = ctx.mlp_get_params()
    p[-48:] = 1e3
    ctx.mlp_set_params(p)
    rho = torch.zeros(s.nblk * o * o, dtype=torch.float64, device="cuda")
    st = torch.zeros(len(cols) * ma.STATS, dtype=torch.int32, device="cuda")
    ctx.solve_columns(cols, s.p, s.q, mu=0.95, kT=s.kT, rho=rho, col_stats=st,
                      opts=ma.default_opts(start="learned"))
    st = st.cpu().numpy().reshape(-1, ma.STATS)
    assert np.all(st[:, 4] == 2)
    assert np.abs(rho.cpu().numpy() - rho_o).max() < 1e-10
    ctx.mlp_init(seed=3)


def test_trained_network_reduces_cg_iterations(env):
    """Train on one 4,096-atom geometry, evaluate on a fresh seed: fewer CG
    iterations at the same rho error (CG tolerance 1e-8, both starts compared
    with the FP64 result at tolerance 1e-12)."""
    torch, ma, ctx, s = env
    from paper_1202_0098_amd import learned
    X, T = learned.collect_pairs(ctx, synth.config_diamond4096(2101))
    ctx.mlp_init(seed=7)
    hist = learned.train(ctx, X, T, epochs=10, batch=256, lr=1e-3)
    _say(f"training loss {hist[0]:.3e} -> {hist[-1]:.3e}")
    assert hist[-1] < 0.5 * hist[0]
    tb = synth.config_diamond4096(2001)
    ctx.build_tb(tb)
    ref = learned.cg_stats(ctx, tb, "zero", cg_tol=1e-12, reps=1, mu=0.95)
    z = learned.cg_stats(ctx, tb, "zero", cg_tol=1e-8, reps=1, mu=0.95)
    l = learned.cg_stats(ctx, tb, "learned", cg_tol=1e-8, reps=1, mu=0.95)
    ez = np.abs(z["rho"] - ref["rho"]).max()
    el = np.abs(l["rho"] - ref["rho"]).max()
    _say(f"CG iterations zero {z['cg_mean']:.2f} learned {l['cg_mean']:.2f}, fallback "
         f"{l['fallback']:.3f}, columns/s {z['cols_per_s']:.4g} -> {l['cols_per_s']:.4g}, "
         f"rho error at CG tol 1e-8: zero {ez:.2e} learned {el:.2e}")
    assert l["cg_mean"] < z["cg_mean"]
    assert l["fallback"] < 0.01
    # equal rho error: both within the CG-tolerance-limited error
    assert ez < 1e-4 and el < 1e-4
    ctx.build_tb(s)
    ctx.mlp_init(seed=3)


def test_c4_protocol_on_a_fresh_disordered_seed(env):
    """The start network's evaluation protocol at test size: train on pairs
    from the 64-atom cell and one 4,096-atom geometry (crystalline), evaluate
    on a fresh seed of the 8,000-atom disordered cell with the CG tolerance at
    1e-8, mixed_f64acc, against the zero start: CG iterations, columns/s and
    the max rho error against the FP64 solve at tolerance 1e-12 for both.
    What holds and is asserted: at CG tolerance 1e-8 both starts stay within
    1e-3 of the FP64 result (with p = q = 20 the block-2 Krylov space
    K_20(H; s_j) amplifies the s_j error the tolerance allows: 7.6e-5 for the
    zero start, 6.0e-4 for the learned one on this seed), and every column
    either uses or rejects its prediction; the numbers are reported.  The
    network does not transfer from crystalline to disordered environments
    well enough to cut the iterations, and at equal CG tolerance its rho
    error is larger (a negative result that the printed numbers record)."""
    torch, ma, ctx, s = env
    from paper_1202_0098_amd import learned
    Xs, Ts = [], []
    for tb in (synth.config_diamond64(1001), synth.config_diamond4096(2101)):
        X, T = learned.collect_pairs(ctx, tb)
        Xs.append(X)
        Ts.append(T)
    X, T = torch.cat(Xs).contiguous(), torch.cat(Ts).contiguous()
    ctx.mlp_init(seed=7)
    hist = learned.train(ctx, X, T, epochs=8, batch=512, lr=1e-3)
    _say(f"{X.shape[0]} pairs, training loss {hist[0]:.3e} -> {hist[-1]:.3e}")
    tb = synth.config_disordered8000(3006)
    ctx.build_tb(tb)
    ref = learned.cg_stats(ctx, tb, "zero", cg_tol=1e-12, precision="fp64", reps=1)
    z = learned.cg_stats(ctx, tb, "zero", cg_tol=1e-8, precision="mixed_f64acc", reps=2,
                         mu=ref["mu"])
    lr_ = learned.cg_stats(ctx, tb, "learned", cg_tol=1e-8, precision="mixed_f64acc", reps=2,
                           mu=ref["mu"])
    ez = float(np.abs(z["rho"] - ref["rho"]).max())
    el = float(np.abs(lr_["rho"] - ref["rho"]).max())
    _say(f"disordered8000 seed 3006: CG iterations zero {z['cg_mean']:.2f} learned "
         f"{lr_['cg_mean']:.2f}; columns/s {z['cols_per_s']:.4g} -> {lr_['cols_per_s']:.4g}; "
         f"predictions used {lr_['learned']:.3f}, rejected {lr_['fallback']:.3f}; max rho error "
         f"zero {ez:.2e} learned {el:.2e}")
    assert ez <= 1e-3 and el <= 1e-3
    assert abs(lr_["learned"] + lr_["fallback"] - 1.0) < 1e-12
    ctx.build_tb(s)
    ctx.mlp_init(seed=3)


def test_training_rejects_an_index_outside_the_table(env):
    """The gather checks the device row indices: an index past the end of
    the table (or negative) fails the training step with MA_EINVAL before
    the parameters change."""
    torch, ma, ctx, s = env
    sh = ctx.mlp_shape()
    n = 64
    rng = np.random.default_rng(21)
    X = torch.from_numpy(rng.normal(size=(n, sh["n_in"])).astype(np.float32)).cuda()
    T = torch.from_numpy((rng.normal(size=(n, sh["n_out"])) * 0.1).astype(np.float32)).cuda()
    p0 = ctx.mlp_get_params()
    for bad in (n, -1):
        idx = torch.arange(32, dtype=torch.int32, device="cuda")
        idx[7] = bad
        with pytest.raises(ma.MarnoldiError) as ei:
            ctx.mlp_train_step(X, T, 32, 1e-3, idx=idx)
        assert ei.value.status == ma.MA_EINVAL
    assert np.array_equal(ctx.mlp_get_params(), p0)
    # in range: accepted
    idx = torch.arange(32, dtype=torch.int32, device="cuda") + 32
    ctx.mlp_train_step(X, T, 32, 1e-3, idx=idx)
    ctx.mlp_init(seed=3)
