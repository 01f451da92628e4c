"""The learned line shape on the GPU against the FP64 oracle.

* forward pass (BF16 weights, split-BF16 activations, MFMA) vs the oracle's
  FP64 network evaluated with the same BF16-rounded weights;
* loss and gradient of the device backward pass vs the oracle's FP64
  backward pass at the same weights;
* training samples: the device targets vs the oracle's Voigt function;
* training lowers the validation error;
* a PT table evaluated with the trained network stays within 1e-3 of the
  oracle's direct sum, and the network cuts the error of its analytic base
  alone (the method without the learned part) by more than tenfold.
"""
import numpy as np
import pytest

import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

WIDTHS = [3, 64, 64, 64, 64, 1]


def M():
    from paper_2411_03418_amd import marfa
    return marfa


def bf16_round(a):
    """Round float32 values to the nearest BF16 (ties to even), as float64."""
    u = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def eval_params(p):
    """The parameters the device evaluates: weights rounded to BF16, biases FP32."""
    q = np.asarray(p, np.float64).copy()
    off = 0
    for i in range(len(WIDTHS) - 1):
        nw = WIDTHS[i] * WIDTHS[i + 1]
        q[off:off + nw] = bf16_round(p[off:off + nw])
        off += nw + WIDTHS[i + 1]
    return q


def random_params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    parts = []
    for i in range(len(WIDTHS) - 1):
        fan = WIDTHS[i] + WIDTHS[i + 1]
        parts.append(rng.uniform(-1, 1, WIDTHS[i] * WIDTHS[i + 1]) * np.sqrt(6.0 / fan) * scale)
        parts.append(rng.uniform(-0.3, 0.3, WIDTHS[i + 1]))
    return np.concatenate(parts).astype(np.float32)


def random_features(n, seed):
    rng = np.random.default_rng(seed)
    return np.stack([rng.uniform(0, 1.8, n), rng.uniform(-2, 1.5, n), rng.uniform(0, 1, n)], 1).astype(np.float32)


def test_forward_matches_oracle_network():
    S = M().Surrogate(chi="tonkov", cutoff=125.0, seed=3)
    p = random_params(11, scale=1.5)
    S.set_params(p)
    X = random_features(1000, 12)   # not a multiple of 64: ragged last wavefront
    got = S.forward(torch.tensor(X, device="cuda:0")).cpu().numpy().astype(np.float64)
    ref = O.mlp_forward(WIDTHS, eval_params(p), X.astype(np.float64))[:, 0]
    err = np.abs(got - ref) / np.maximum(1.0, np.abs(ref))
    print(f"forward: max err {err.max():.2e}, output range {ref.min():.3f} .. {ref.max():.3f}")
    assert err.max() < 5e-5
    S.close()


def test_params_round_trip():
    S = M().Surrogate(seed=5)
    p = random_params(13)
    S.set_params(p)
    assert np.array_equal(S.get_params(), p)
    S.close()


def _grad_tolerance(p, X, T):
    """Per-parameter bound on the device gradient's error.  The oracle's
    per-sample gradients c_b (batch of one, divided by n) give
    A = sum_b |c_b|, the sum of the magnitudes the device accumulates.  The
    device forms the hidden-layer weight gradients as matrix-core products of
    BF16-rounded dZ and H (two roundings of at most 2^-9 each per product:
    2^-8 A), everything else in single precision (1e-5 A)."""
    n = X.shape[0]
    A = np.zeros(p.size)
    for b in range(n):
        _, gb = O.mlp_loss_grad(WIDTHS, eval_params(p), X[b:b + 1].astype(np.float64),
                                T[b:b + 1].astype(np.float64))
        A += np.abs(gb) / n
    rel = np.full(p.size, 1e-5)
    off = 0
    for i in range(len(WIDTHS) - 1):
        nw = WIDTHS[i] * WIDTHS[i + 1]
        if 1 <= i <= 3:
            rel[off:off + nw] += 2.0 ** -8
        off += nw + WIDTHS[i + 1]
    return rel * A + 1e-12 * A.max()


@pytest.mark.parametrize("targets", ["random", "offset"])
def test_gradient_matches_oracle_elementwise(targets):
    S = M().Surrogate(seed=3)
    p = random_params(21)
    S.set_params(p)
    n = 1000   # 31 full groups of 32 samples and a ragged one
    X = random_features(n, 22)
    rng = np.random.default_rng(23)
    if targets == "random":
        T = rng.normal(0, 0.5, n).astype(np.float32)
    else:
        # every error between 1 and 1.2: little cancellation between samples
        t = O.mlp_forward(WIDTHS, eval_params(p), X.astype(np.float64))[:, 0]
        T = (t - 1.0 - 0.2 * rng.uniform(0, 1, n)).astype(np.float32)
    loss, g = S.loss_grad(torch.tensor(X, device="cuda:0"), torch.tensor(T, device="cuda:0"))
    ref_loss, ref_g = O.mlp_loss_grad(WIDTHS, eval_params(p), X.astype(np.float64), T.astype(np.float64))
    print(f"loss {loss:.6e} vs {ref_loss:.6e}")
    assert abs(loss - ref_loss) <= 1e-4 * ref_loss
    tol = _grad_tolerance(p, X, T)
    err = np.abs(g.astype(np.float64) - ref_g)
    worst = int(np.argmax(err / tol))
    print(f"gradient: max |err|/tol {err[worst] / tol[worst]:.3f} at parameter {worst}; "
          f"max rel err {np.max(err / np.maximum(np.abs(ref_g), 1e-30)):.2e}")
    assert np.all(err <= tol), np.flatnonzero(err > tol)[:20]
    # the bound is tight enough that a sign error in almost any entry exceeds it
    caught = float(np.mean(2.0 * np.abs(ref_g) > tol))
    print(f"entries whose sign flip the bound catches: {caught:.4f}")
    assert caught > 0.9
    S.close()


def test_training_samples_match_oracle_voigt():
    S = M().Surrogate(chi="tonkov", cutoff=125.0, seed=3)
    X, T = S.make_samples(20000, seed=99)
    X = X.cpu().numpy().astype(np.float64)
    T = T.cpu().numpy().astype(np.float64)
    x = np.sinh(8.0 * X[:, 0])
    y = 10.0 ** (2.0 * X[:, 1])
    ad = 3.0 + 125.0 * X[:, 2]
    chi = np.where(X[:, 2] > 0, np.array([O.chi(1, a) for a in ad]), 1.0)
    r = x * x + y * y
    kb = (y * (1 + (3 * x * x - y * y) / (2 * r * r + 1)) / (np.sqrt(np.pi) * (r + 0.5 * np.exp(-r)))
          + np.exp(-x * x) / (1 + np.sqrt(np.pi) * y) ** 2)
    ref = np.log(O.voigt_K(x, y) * chi) - np.log(kb)
    # features are single precision: x carries ~1e-6 relative rounding
    err = np.abs(T - ref)
    print(f"targets: max |dt| {err.max():.2e}; y {y.min():.2e} .. {y.max():.2e}; x up to {x.max():.2e}")
    assert err.max() < 3e-5
    assert y.min() >= 0.99e-4 and y.max() <= 1.01e3
    S.close()


def test_training_reduces_validation_error():
    S = M().Surrogate(chi="tonkov", cutoff=125.0, seed=3)
    Xv, Tv = S.make_samples(50000, seed=7)
    before = (S.forward(Xv) - Tv).abs().max().item()
    rep = S.train(n_train=200_000, n_val=50_000, epochs=3, batch=4096, lr_max=2e-3, lr_min=1e-4, seed=8)
    after = (S.forward(Xv) - Tv).abs().max().item()
    print(f"train report {rep}; max |dt| before {before:.3f}, after {after:.3f}")
    assert rep["steps"] == 3 * (200_000 // 4096)
    assert after < 0.5 * before
    S.close()


def _rel(got, ref):
    m = ref >= 1e-8 * ref.max()
    return float(np.max(np.abs(got[m] - ref[m]) / ref[m]))


def test_surrogate_pt_table_vs_direct_and_vs_base_alone():
    from paper_2411_03418_amd import synth
    mm = M()
    lines = synth.make_lines(3000, 930.0, 1090.0, 41, shift=True)
    layers = synth.pt_table(7)
    req = dict(nu_begin=1000.0, nu_end=1013.5, cutoff=60.0, chi="tonkov", prune=1e-6)
    S = mm.Surrogate(chi="tonkov", cutoff=60.0, seed=1)
    rep = S.fit(nu_lo=925.0, nu_hi=1095.0, T_lo=150.0, T_hi=740.0)
    print(f"fit: {rep}")
    plan = mm.Plan(lines, layers, device=0, **req)
    plain = plan.execute().clone()
    plan.set_surrogate(S)
    plan.set_eval("surrogate")
    surr = plan.execute().clone()
    S.set_params(np.zeros(mm.N_PARAMS, np.float32))   # t = 0: the analytic base alone
    base = plan.execute().clone()
    torch.cuda.synchronize()
    plan.close()
    rng = np.random.default_rng(5)
    m0 = int(req["nu_begin"] * 2048)
    nodes = np.unique(np.concatenate([rng.integers(m0, int(req["nu_end"] * 2048) + 1, 1500),
                                      np.arange(m0 + 6000, m0 + 6400)]))
    o = dict(nu_begin=req["nu_begin"], nu_end=req["nu_end"], cutoff=req["cutoff"], chi=1, prune=req["prune"])
    e_s, e_b, e_p = [], [], []
    for i in range(layers.shape[0]):
        ref = O.direct(lines, layers[i], nodes, threads=16, **o)
        e_s.append(_rel(surr[i, nodes - m0].double().cpu().numpy(), ref))
        e_b.append(_rel(base[i, nodes - m0].double().cpu().numpy(), ref))
        e_p.append(_rel(plain[i, nodes - m0].double().cpu().numpy(), ref))
    print(f"vs direct: plain {max(e_p):.2e}, surrogate {max(e_s):.2e}, base alone {max(e_b):.2e}")
    full = max(_rel(surr[i].double().cpu().numpy(), plain[i].double().cpu().numpy()) for i in range(layers.shape[0]))
    print(f"surrogate vs plain, every node: {full:.2e}")
    assert max(e_s) < 1e-3
    assert max(e_b) > 10 * max(e_s)
    S.close()


def test_surrogate_eval_switch_and_set_params_after_execute():
    """The request's eval field selects the line shape, and replacing the
    network's weights right after an execute (no synchronisation in between)
    leaves that execute's output computed with the old weights."""
    from paper_2411_03418_amd import synth
    mm = M()
    lines = synth.make_lines(2000, 940.0, 1080.0, 43, shift=True)
    layers = synth.pt_table(4)
    req = dict(nu_begin=1000.0, nu_end=1012.0, cutoff=60.0, chi="tonkov", prune=1e-6)
    S = mm.Surrogate(chi="tonkov", cutoff=60.0, seed=2)
    S.train(n_train=65536, n_val=4096, epochs=2, batch=4096, lr_max=2e-3, lr_min=1e-4, seed=9,
            nu_lo=935.0, nu_hi=1085.0, T_lo=150.0, T_hi=740.0)
    trained = S.get_params()
    # a plan asking for the learned shape refuses to run until one is attached
    plan = mm.Plan(lines, layers, device=0, eval="surrogate", **req)
    with pytest.raises(mm.MarfaError) as e:
        plan.execute()
    assert e.value.status == mm.E_UNSUPPORTED
    plan.set_surrogate(S)
    ref = plan.execute().clone()
    torch.cuda.synchronize()
    # plain evaluation with the network still attached ignores it
    plan.set_eval("plain")
    plain = plan.execute().clone()
    torch.cuda.synchronize()
    assert not torch.equal(plain, ref)
    plan.set_eval("surrogate")
    again = plan.execute().clone()
    torch.cuda.synchronize()
    assert torch.equal(again, ref)
    # weights replaced while the execute may still be running
    out = plan.execute()
    S.set_params(np.zeros(mm.N_PARAMS, np.float32))
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    base = plan.execute().clone()
    torch.cuda.synchronize()
    assert not torch.equal(base, ref)
    S.set_params(trained)
    back = plan.execute().clone()
    torch.cuda.synchronize()
    assert torch.equal(back, ref)
    plan.close()
    S.close()


def test_surrogate_save_load_round_trip(tmp_path):
    """A network saved after training and loaded into a new handle attaches to
    a plan and gives the same output, bit for bit; an untrained network has
    nothing to save and a load needs a positive x_max."""
    from paper_2411_03418_amd import synth
    mm = M()
    lines = synth.make_lines(1500, 950.0, 1070.0, 47, shift=True)
    layers = synth.pt_table(3)
    req = dict(nu_begin=1000.0, nu_end=1008.0, cutoff=60.0, chi="tonkov", prune=1e-6)
    S = mm.Surrogate(chi="tonkov", cutoff=60.0, seed=3)
    with pytest.raises(mm.MarfaError) as e:
        S.save(str(tmp_path / "untrained.npz"))
    assert e.value.status == mm.E_UNSUPPORTED
    rep = S.train(n_train=65536, n_val=4096, epochs=2, batch=4096, lr_max=2e-3, lr_min=1e-4, seed=11,
                  nu_lo=945.0, nu_hi=1075.0, T_lo=150.0, T_hi=740.0)
    path = str(tmp_path / "net.npz")
    S.save(path)
    plan = mm.Plan(lines, layers, device=0, eval="surrogate", **req)
    plan.set_surrogate(S)
    ref = plan.execute().clone()
    torch.cuda.synchronize()
    plan.set_surrogate(None)
    S.close()
    L = mm.Surrogate.load(path)
    with np.load(path) as z:
        assert float(z["x_max"]) == rep["x_max"]
        assert np.array_equal(L.get_params(), z["params"])
        params = np.ascontiguousarray(z["params"], np.float32)
        for bad in (0.0, -1.0, float("inf"), float("nan")):
            assert mm.lib().marfa_surrogate_load(L._h, mm._ptr(params), mm.N_PARAMS, bad) == mm.E_INVALID
    plan.set_surrogate(L)
    got = plan.execute().clone()
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    plan.close()
    L.close()
