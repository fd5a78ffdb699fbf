"""GPU parity of F(X|Theta) (hash grid + MLP + four heads, Sec. III-C) against the
float64 PyTorch oracle: parameters, and the gradients of every table and weight."""
import numpy as np
import pytest
import torch

from oracle import ngp as N
from paper_2403_11577_amd import binding as B

from gpu_util import rel_close, say

pytestmark = pytest.mark.gpu

CONFIGS = {
    "default": N.NgpConfig(),
    "small_hashed": N.NgpConfig(levels=4, feat=2, log2_table=10, n_min=4, n_max=64, hidden=64, scale_max=0.2),
}


def _case(cfg, G, seed):
    rng = np.random.default_rng(seed)
    lo, hi = np.array([-20.0, -5.0, -1.0]), np.array([30.0, 15.0, 4.0])
    x = rng.uniform(lo, hi, size=(G, 3))
    x[:5] = [lo, hi, (lo + hi) / 2, lo - 1.0, hi + 2.0]      # box corners, centre, outside (clamped)
    m = N.init_model(cfg, seed=seed)
    m["tables"] = rng.uniform(-0.5, 0.5, size=m["tables"].shape).astype(np.float32)
    m["b1"] = rng.uniform(-0.1, 0.1, size=m["b1"].shape).astype(np.float32)
    m["b3"] = rng.uniform(-0.5, 0.5, size=m["b3"].shape).astype(np.float32)
    return x.astype(np.float32), lo, hi, m


def _kink_free(cfg, x, lo, hi, m, rel=1e-5):
    """Gaussians whose hidden pre-activations all lie clear of the ReLU kink.  The kernel
    takes each ReLU decision in float32 and the oracle in float64; a pre-activation within
    float32 rounding of zero (|pre| <= rel * the sum of its terms' magnitudes) may be decided
    either way, both correct, so such Gaussians are left out of gradient comparisons (their
    output gradients are zero on both sides)."""
    import torch as _t
    t = {k: _t.tensor(np.asarray(v, np.float64)) for k, v in m.items()}
    enc = N.encode(cfg, np.asarray(x, np.float64), lo, hi, t["tables"])
    p1 = enc @ t["w1"].T + t["b1"]
    s1 = enc.abs() @ t["w1"].abs().T + t["b1"].abs()
    h1 = _t.relu(p1)
    p2 = h1 @ t["w2"].T + t["b2"]
    s2 = h1 @ t["w2"].abs().T + t["b2"].abs()
    return ((p1.abs() > rel * s1).all(dim=1) & (p2.abs() > rel * s2).all(dim=1)).numpy()


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def _gpu_model(cfg, lo, hi, m):
    t = {k: _dev(v) for k, v in m.items()}
    return t, B.ngp_struct(cfg, lo, hi, t["tables"], t["w1"], t["b1"], t["w2"], t["b2"], t["w3"], t["b3"])


@pytest.mark.parametrize("name", list(CONFIGS))
def test_ngp_forward_vs_oracle(name):
    cfg = CONFIGS[name]
    say(f"case: ngp forward {name}")
    x, lo, hi, m = _case(cfg, 4000, 1)
    t, model = _gpu_model(cfg, lo, hi, m)
    G = x.shape[0]
    xs = _dev(x.T)
    out = dict(quat=torch.empty((4, G), device="cuda"), scale=torch.empty((3, G), device="cuda"),
               opacity=torch.empty(G, device="cuda"), color=torch.empty((3, G), device="cuda"))
    B.splat_ngp_fwd(model, xs, out["quat"], out["scale"], out["opacity"], out["color"])
    torch.cuda.synchronize()
    ref = N.params(cfg, x.astype(np.float64), lo, hi, m)
    for k in out:
        a = out[k].cpu().numpy().astype(np.float64)
        err = np.abs(a - ref[k]).max() / max(1e-30, np.abs(ref[k]).max())
        say(f"  {k}: max err / max {err:.2e}")
        assert err <= 2e-5, k


@pytest.mark.parametrize("name", list(CONFIGS))
def test_ngp_backward_vs_oracle(name):
    cfg = CONFIGS[name]
    say(f"case: ngp backward {name}")
    x, lo, hi, m = _case(cfg, 3000, 2)
    t, model = _gpu_model(cfg, lo, hi, m)
    G = x.shape[0]
    rng = np.random.default_rng(3)
    d = dict(quat=rng.normal(size=(4, G)), scale=rng.normal(size=(3, G)), opacity=rng.normal(size=G),
             color=rng.normal(size=(3, G)))
    keep = _kink_free(cfg, x, lo, hi, m)
    d = {k: v * keep for k, v in d.items()}
    dd = {k: _dev(v.astype(np.float32)) for k, v in d.items()}
    grads = {k: torch.zeros_like(v) for k, v in t.items()}
    ws = torch.empty(B.splat_ngp_workspace_size(G), dtype=torch.uint8, device="cuda")
    B.splat_ngp_bwd(model, _dev(x.T), dd["quat"], dd["scale"], dd["opacity"], dd["color"], ws, grads["tables"],
                    grads["w1"], grads["b1"], grads["w2"], grads["b2"], grads["w3"], grads["b3"])
    torch.cuda.synchronize()
    d32 = {k: v.astype(np.float32).astype(np.float64) for k, v in d.items()}
    _, ref = N.params_and_grads(cfg, x.astype(np.float64), lo, hi, m, d32)
    for k in ("w3", "b3", "w2", "b2", "w1", "b1", "tables"):
        ok, err = rel_close(grads[k].cpu().numpy(), ref[k], 1e-3)
        say(f"  {k}: {err:.2e}")
        assert ok, (k, err)


def _bwd(model, xs, dd, ws, grads, index=None):
    if index is None:
        B.splat_ngp_bwd(model, xs, dd["quat"], dd["scale"], dd["opacity"], dd["color"], ws, grads["tables"],
                        grads["w1"], grads["b1"], grads["w2"], grads["b2"], grads["w3"], grads["b3"])
    else:
        B.splat_ngp_bwd_indexed(model, xs, index, dd["quat"], dd["scale"], dd["opacity"], dd["color"], ws,
                                grads["tables"], grads["w1"], grads["b1"], grads["w2"], grads["b2"], grads["w3"],
                                grads["b3"])


def _index(model, xs):
    G = xs.shape[1]
    index = torch.empty(B.splat_ngp_index_size(model, G), dtype=torch.uint8, device="cuda")
    bws = torch.empty(B.splat_ngp_index_workspace_size(model, G), dtype=torch.uint8, device="cuda")
    B.splat_ngp_index_build(model, xs, index, bws)
    return index


@pytest.mark.parametrize("name", list(CONFIGS))
@pytest.mark.parametrize("G", [5, 3000, 66001])
def test_ngp_indexed_backward_vs_oracle_and_reproducible(name, G):
    """Table gradients through the inverse index: the oracle's to 1e-3, the same weight
    gradients as the atomic path bit for bit, and the same result on every call.  At 66,001
    Gaussians every workgroup of the weight-gradient products walks more than one batch of
    64 and the last range ends inside a 16-byte quad."""
    cfg = CONFIGS[name]
    say(f"case: ngp indexed backward {name} G={G}")
    x, lo, hi, m = _case(cfg, max(G, 5), 4)
    x = x[:G]
    t, model = _gpu_model(cfg, lo, hi, m)
    rng = np.random.default_rng(5)
    d = dict(quat=rng.normal(size=(4, G)), scale=rng.normal(size=(3, G)), opacity=rng.normal(size=G),
             color=rng.normal(size=(3, G)))
    d["opacity"][::3] = 0.0
    keep = _kink_free(cfg, x, lo, hi, m)
    say(f"  {int((~keep).sum())} of {G} Gaussians within float32 rounding of a ReLU kink left out")
    d = {k: v * keep for k, v in d.items()}
    dd = {k: _dev(v.astype(np.float32)) for k, v in d.items()}
    xs = _dev(x.T)
    ws = torch.empty(B.splat_ngp_workspace_size(G), dtype=torch.uint8, device="cuda")
    index = _index(model, xs)
    runs = []
    for _ in range(2):
        grads = {k: torch.zeros_like(v) for k, v in t.items()}
        _bwd(model, xs, dd, ws, grads, index)
        torch.cuda.synchronize()
        runs.append({k: v.cpu().numpy() for k, v in grads.items()})
    for k in runs[0]:
        assert np.array_equal(runs[0][k], runs[1][k]), k
    scat = {k: torch.zeros_like(v) for k, v in t.items()}
    _bwd(model, xs, dd, ws, scat)
    torch.cuda.synchronize()
    for k in ("w1", "b1", "w2", "b2", "w3", "b3"):
        assert np.array_equal(runs[0][k], scat[k].cpu().numpy()), k
    d32 = {k: v.astype(np.float32).astype(np.float64) for k, v in d.items()}
    _, ref = N.params_and_grads(cfg, x.astype(np.float64), lo, hi, m, d32)
    for k in ("tables", "w1", "b1", "w2", "b2", "w3", "b3"):
        ok, err = rel_close(runs[0][k], ref[k], 1e-3)
        say(f"  {k}: {err:.2e}")
        assert ok, (k, err)
    ok, err = rel_close(runs[0]["tables"], scat["tables"].cpu().numpy(), 1e-4)
    assert ok, err


def test_ngp_indexed_backward_at_two_million_gaussians():
    """The drive scene's 2 M means, default grid: the indexed table gradient agrees with
    the atomic one (float rounding apart) and is added to what dtables held."""
    import synth
    say("case: ngp indexed backward, 2M Gaussians")
    pts = synth.batched64(seed=0).gauss.mean.astype(np.float64)
    G = pts.shape[1]
    cfg = CONFIGS["default"]
    lo, hi = pts.min(axis=1) - 1.0, pts.max(axis=1) + 1.0
    m = N.init_model(cfg, seed=7)
    rng = np.random.default_rng(8)
    m["tables"] = rng.uniform(-0.5, 0.5, size=m["tables"].shape).astype(np.float32)
    t, model = _gpu_model(cfg, lo, hi, m)
    xs = _dev(pts.astype(np.float32))
    g = torch.Generator(device="cpu").manual_seed(9)
    dd = {k: (torch.randn(s, generator=g) * 1e-3).to("cuda") for k, s in
          (("quat", (4, G)), ("scale", (3, G)), ("opacity", (G,)), ("color", (3, G)))}
    dd["opacity"][G // 2:] = 0.0
    ws = torch.empty(B.splat_ngp_workspace_size(G), dtype=torch.uint8, device="cuda")
    index = _index(model, xs)
    gi = {k: torch.zeros_like(v) for k, v in t.items()}
    _bwd(model, xs, dd, ws, gi, index)
    gs = {k: torch.zeros_like(v) for k, v in t.items()}
    _bwd(model, xs, dd, ws, gs)
    # every row is written once, so onto a non-zero start the result is start + gradient in float32
    base = torch.randn(t["tables"].shape, generator=g).to("cuda")
    gb = base.clone()
    gw = {k: torch.zeros_like(v) for k, v in t.items()}
    gw["tables"] = gb
    _bwd(model, xs, dd, ws, gw, index)
    torch.cuda.synchronize()
    a = gi["tables"].cpu().numpy()
    b = gs["tables"].cpu().numpy()
    # the atomic path adds up to 9,000 float32 terms per row in an order that varies between runs
    # (worst case k u = 5.4e-4 of the row's absolute-term sum): element-wise the parity metric,
    # over the whole tensor 1e-4
    ok, err = rel_close(a, b, 1e-3)
    tens = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    say(f"  tables vs atomics: {err:.2e} (tensor {tens:.2e})")
    assert ok, err
    assert tens <= 1e-4, tens
    assert np.array_equal(gb.cpu().numpy(), base.cpu().numpy() + a)
    for k in ("w1", "b1", "w2", "b2", "w3", "b3"):
        assert torch.equal(gi[k], gs[k]), k


@pytest.mark.parametrize("name", list(CONFIGS))
def test_ngp_training_forward_and_saved_adjoint(name):
    """The training forward gives the forward's parameters bit for bit, and the adjoint from
    its stored values equals the adjoint that evaluates the field again, on every call."""
    cfg = CONFIGS[name]
    say(f"case: ngp training forward / saved adjoint {name}")
    x, lo, hi, m = _case(cfg, 2500, 6)
    t, model = _gpu_model(cfg, lo, hi, m)
    G = x.shape[0]
    xs = _dev(x.T)
    mk = lambda: dict(quat=torch.empty((4, G), device="cuda"), scale=torch.empty((3, G), device="cuda"),
                      opacity=torch.empty(G, device="cuda"), color=torch.empty((3, G), device="cuda"))
    a, b = mk(), mk()
    ws = torch.empty(B.splat_ngp_workspace_size(G), dtype=torch.uint8, device="cuda")
    B.splat_ngp_fwd(model, xs, a["quat"], a["scale"], a["opacity"], a["color"])
    B.splat_ngp_fwd_train(model, xs, b["quat"], b["scale"], b["opacity"], b["color"], ws)
    torch.cuda.synchronize()
    for k in a:
        assert torch.equal(a[k], b[k]), k
    rng = np.random.default_rng(7)
    dd = {k: _dev(rng.normal(size=v.shape).astype(np.float32)) for k, v in a.items()}
    index = _index(model, xs)
    ref = {k: torch.zeros_like(v) for k, v in t.items()}
    ws2 = torch.empty_like(ws)
    _bwd(model, xs, dd, ws2, ref, index)
    for _ in range(2):
        got = {k: torch.zeros_like(v) for k, v in t.items()}
        B.splat_ngp_bwd_saved(model, G, index, dd["quat"], dd["scale"], dd["opacity"], dd["color"], ws,
                              got["tables"], got["w1"], got["b1"], got["w2"], got["b2"], got["w3"], got["b3"])
        torch.cuda.synchronize()
        for k in ref:
            assert torch.equal(got[k], ref[k]), k
