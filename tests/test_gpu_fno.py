"""Warm-start network on the GPU against its float64 reference: forward outputs, losses,
gradients and the Adam step, through the C ABI (libgsi.so, include/fno.h)."""
import numpy as np
import pytest

from oracle import fno_oracle as F

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

SMALL = F.Config(N=16, m=6, w=5, L=2, p=4)


def _net(cfg, B, seed=0, bf16=False):
    from paper_2306_10379_amd import fno
    return fno.Net(N=cfg.N, modes=cfg.m, width=cfg.w, layers=cfg.L, p=cfg.p, max_batch=B, seed=seed,
                   bf16_weights=bf16)


def _case(cfg, B, seed, scale=0.3):
    g = np.random.default_rng(seed)
    flat = scale * g.standard_normal(F.param_count(cfg))
    V = -20.0 * g.random((B, cfg.N * cfg.N))
    Xs = np.stack([np.linalg.qr(g.standard_normal((cfg.N * cfg.N, cfg.p)))[0] for _ in range(B)])
    return flat, V, Xs


def _dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


@pytest.mark.parametrize("cfg", [SMALL, F.Config(N=32, m=11, w=7, L=3, p=9)], ids=["N16", "N32"])
def test_forward_loss_and_gradient_match_reference(cfg):
    B = 3
    flat, V, Xs = _case(cfg, B, 7)
    net = _net(cfg, B)
    print(f"fno {cfg} params {net.count}", flush=True)
    assert net.count == F.param_count(cfg)
    # the reference sees the float32-rounded parameters and inputs the device uses
    flat32, V32, X32 = (np.asarray(a, np.float32).astype(np.float64) for a in (flat, V, Xs))
    net.set_params(_dev(flat))
    Y = net.forward(_dev(V)).double().cpu().numpy()
    Yref = F.predict(flat32, V32, cfg)
    assert np.max(np.abs(Y - Yref)) <= 2e-5 * np.max(np.abs(Yref))
    loss, grad = net.loss_grad(_dev(V), _dev(Xs))
    lref, gref, per = F.loss_and_grad(flat32, V32, X32, cfg)
    assert np.allclose(loss, per, rtol=1e-4, atol=1e-5)
    g = grad.double().cpu().numpy()
    # every parameter group: max deviation relative to the group's largest entry
    off = 0
    for name, shape in F.param_shapes(cfg):
        size = int(np.prod(shape))
        ref = gref[off:off + size]
        assert np.max(np.abs(g[off:off + size] - ref)) <= 1e-3 * np.max(np.abs(ref)) + 1e-7, name
        off += size
    net.close()


def test_full_size_network_matches_reference():
    """The warm-start network at its working size: 256 x 256 grid, 24 x 24 modes, width 20,
    4 hidden layers, 32 outputs (1.29M parameters), batch of 2. The loss gradient carries
    (Y^T Y)^-1, so float32 rounding in Y is amplified by cond(Y^T Y): the case is drawn with
    well-spread weights (cond printed) and the bound is 2e-3 of each group's largest entry."""
    cfg = F.Config()
    B = 2
    flat, V, Xs = _case(cfg, B, 11, scale=0.3)
    net = _net(cfg, B)
    flat32, V32, X32 = (np.asarray(a, np.float32).astype(np.float64) for a in (flat, V, Xs))
    net.set_params(_dev(flat))
    loss, grad = net.loss_grad(_dev(V), _dev(Xs))
    lref, gref, per = F.loss_and_grad(flat32, V32, X32, cfg)
    Yref = F.predict(flat32, V32, cfg)
    conds = [np.linalg.cond(Yb.T @ Yb) for Yb in Yref]
    print(f"full size: loss {loss} reference {per}, cond(Y^T Y) {conds}", flush=True)
    assert np.allclose(loss, per, rtol=1e-4, atol=1e-4)
    g = grad.double().cpu().numpy()
    off = 0
    for name, shape in F.param_shapes(cfg):
        size = int(np.prod(shape))
        ref = gref[off:off + size]
        assert np.max(np.abs(g[off:off + size] - ref)) <= 2e-3 * np.max(np.abs(ref)) + 1e-7, name
        off += size
    net.close()


def test_adam_step_matches_reference():
    cfg = SMALL
    B = 2
    flat, V, Xs = _case(cfg, B, 5)
    net = _net(cfg, B)
    net.set_params(_dev(flat))
    w = np.asarray(flat, np.float32).astype(np.float64)
    m, v = np.zeros_like(w), np.zeros_like(w)
    for t in (1, 2, 3):
        net.set_params(_dev(w))
        _, grad = net.loss_grad(_dev(V), _dev(Xs))
        gcpu = grad.double().cpu().numpy()
        net.adam(1e-3)
        F.adam_step(w, gcpu, m, v, t, lr=1e-3)
        got = net.get_params().double().cpu().numpy()
        assert np.max(np.abs(got - w)) <= 1e-6 + 1e-5 * np.max(np.abs(w))
        w = got.copy()
    net.close()


def _group_max_dev(g, gref, cfg, rel):
    off = 0
    for name, shape in F.param_shapes(cfg):
        size = int(np.prod(shape))
        ref = gref[off:off + size]
        assert np.max(np.abs(g[off:off + size] - ref)) <= rel * np.max(np.abs(ref)) + 1e-7, name
        off += size


@pytest.mark.parametrize("cfg", [SMALL, F.Config(N=32, m=11, w=7, L=3, p=9)], ids=["N16", "N32"])
def test_bf16_weights_match_reference_at_the_rounded_weights(cfg):
    """bfloat16 weights: forward outputs, losses and the gradient equal the float64 reference
    evaluated at the bfloat16-rounded parameters (oracle round_bf16) within the float32 bounds
    of the float32-weight test: both sides use the same rounded weights, so only the float32
    activations and sums differ. The outputs at the unrounded weights lie far outside that
    bound (the device does read the rounded copy), and the master stays unrounded."""
    B = 3
    flat, V, Xs = _case(cfg, B, 7)
    net = _net(cfg, B, bf16=True)
    flat32 = np.asarray(flat, np.float32)
    wb = F.round_bf16(flat32)
    V32, X32 = (np.asarray(a, np.float32).astype(np.float64) for a in (V, Xs))
    net.set_params(_dev(flat))
    assert np.array_equal(net.get_params().cpu().numpy(), flat32)
    Y = net.forward(_dev(V)).double().cpu().numpy()
    Yref = F.predict(wb, V32, cfg)
    bound = 2e-5 * np.max(np.abs(Yref))
    err = np.max(np.abs(Y - Yref))
    far = np.max(np.abs(F.predict(flat32.astype(np.float64), V32, cfg) - Yref))
    print(f"bf16 {cfg}: forward error {err:.2e}, bound {bound:.2e}, unrounded-weight difference {far:.2e}", flush=True)
    assert err <= bound and far > 5 * bound
    loss, grad = net.loss_grad(_dev(V), _dev(Xs))
    lref, gref, per = F.loss_and_grad(wb, V32, X32, cfg)
    assert np.allclose(loss, per, rtol=1e-4, atol=1e-5)
    _group_max_dev(grad.double().cpu().numpy(), gref, cfg, 1e-3)
    net.close()


def test_bf16_adam_updates_the_float32_master():
    """Adam in bfloat16 mode moves the float32 master as in float32 mode (steps of 1e-5, far
    below a bfloat16 ulp of the weights, still accumulate), and the next forward pass reads
    the master rounded to bfloat16."""
    cfg = SMALL
    B = 2
    flat, V, Xs = _case(cfg, B, 5)
    net = _net(cfg, B, bf16=True)
    w = np.asarray(flat, np.float32).astype(np.float64)
    net.set_params(_dev(w))
    m, v = np.zeros_like(w), np.zeros_like(w)
    V32 = np.asarray(V, np.float32).astype(np.float64)
    X32 = np.asarray(Xs, np.float32).astype(np.float64)
    w0 = w.copy()
    for t in (1, 2, 3):
        _, grad = net.loss_grad(_dev(V), _dev(Xs))
        gref = F.loss_and_grad(F.round_bf16(w), V32, X32, cfg)[1]
        _group_max_dev(grad.double().cpu().numpy(), gref, cfg, 1e-3)
        net.adam(1e-5)
        F.adam_step(w, grad.double().cpu().numpy(), m, v, t, lr=1e-5)
        got = net.get_params().double().cpu().numpy()
        assert np.max(np.abs(got - w)) <= 1e-8 + 1e-6 * np.max(np.abs(w))
        w = got.copy()
    assert np.max(np.abs(w - w0)) > 2e-5  # three steps of ~1e-5 each accumulated in the master
    Y = net.forward(_dev(V)).double().cpu().numpy()
    Yref = F.predict(F.round_bf16(w), V32, cfg)
    assert np.max(np.abs(Y - Yref)) <= 2e-5 * np.max(np.abs(Yref))
    net.close()
