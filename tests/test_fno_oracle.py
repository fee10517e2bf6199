"""Pins of the float64 neural-operator reference against facts that do not come from it:
the library sine transform, closed-form reproduction of sine modes, the library's principal
angles, the normal distribution function, central differences, and the Adam paper's first
steps."""
import numpy as np
import pytest
import scipy.fft
import scipy.linalg
import scipy.special
import torch

from oracle import fno_oracle as F

TINY = F.Config(N=12, m=5, w=3, L=2, p=4)


def _rand_params(cfg, seed, scale=0.3):
    g = np.random.default_rng(seed)
    return scale * g.standard_normal(F.param_count(cfg))


def test_param_count_of_the_full_network():
    # width 20, 24 x 24 modes, 4 hidden layers, 32 outputs: about 1.3M parameters
    cfg = F.Config()
    assert F.param_count(cfg) == 20 * 3 + 20 + 4 * (20 * 20 * 24 * 24 + 400 + 20) + 32 * 20 * 576 + 640 + 32
    assert 1.0e6 < F.param_count(cfg) < 1.5e6


def test_sine_basis_is_the_library_dst1_and_orthonormal():
    N, m = 17, 7
    S = F.sine_basis(N, m).numpy()
    x = np.random.default_rng(0).standard_normal(N)
    ref = scipy.fft.dst(x, type=1, norm="ortho")[:m]
    assert np.allclose(S @ x, ref, atol=1e-13)
    assert np.allclose(S @ S.T, np.eye(m), atol=1e-13)


def test_spectral_layer_reproduces_low_sine_modes():
    # with R[o, c] = delta_oc on every mode, K is the projection onto the first m x m sine
    # modes: a product of two low sine modes passes unchanged, a high one is removed
    N, m = 16, 5
    S = F.sine_basis(N, m)
    t = torch.arange(1, N + 1, dtype=torch.float64) / (N + 1)
    low = torch.sin(2 * np.pi * t)[:, None] * torch.sin(4 * np.pi * t)[None, :]
    high = torch.sin(9 * np.pi * t)[:, None] * torch.sin(np.pi * t)[None, :]
    U = torch.stack([low, high])[None]  # (1, 2, N, N)
    R = torch.zeros(2, 2, m, m, dtype=torch.float64)
    R[0, 0] = 1.0
    R[1, 1] = 1.0
    out = F.spectral(U, R, S)
    assert torch.allclose(out[0, 0], low, atol=1e-12)
    assert torch.allclose(out[0, 1], torch.zeros_like(high), atol=1e-12)


def test_gelu_is_t_times_normal_cdf():
    t = torch.linspace(-5, 5, 101, dtype=torch.float64)
    assert np.allclose(F.gelu(t).numpy(), t.numpy() * scipy.special.ndtr(t.numpy()), atol=1e-14)


def test_features_order_matches_the_operator_grid():
    # row-major nodes: x varies along a row, y down the rows, both (i+1)/(N+1)
    N = 5
    V = torch.arange(N * N, dtype=torch.float64)[None]
    f = F.features(V, N)[0]
    assert f[0, 1, 2] == V[0, 1 * N + 2] / 20.0
    assert f[1, 3, 2] == pytest.approx(3.0 / 6.0) and f[2, 3, 2] == pytest.approx(4.0 / 6.0)


def test_zero_network_outputs_the_prior_plus_output_bias():
    cfg = TINY
    flat = np.zeros(F.param_count(cfg))
    bo = np.arange(1, cfg.p + 1, dtype=np.float64)
    flat[-cfg.p:] = bo
    V = np.random.default_rng(1).standard_normal((2, cfg.N * cfg.N))
    Y = F.predict(flat, V, cfg)
    Phi = F.as_blocks(F.prior(cfg.N, cfg.p)[None])[0].numpy()
    assert np.allclose(Y, (Phi + bo)[None])


def test_prior_is_the_lowest_eigenvectors_of_the_grid_laplacian():
    # the p prior columns are eigenvectors of the 5-point Dirichlet Laplacian whose
    # eigenvalues are its p smallest (closed form 4/h^2 (sin^2(k pi h/2) + sin^2(l pi h/2)))
    from paper_2306_10379_amd import inputs as I
    N, p = 14, 11
    A = I.laplacian_2d(N).to_dense() * (N + 1) ** 2
    Phi = F.as_blocks(F.prior(N, p)[None])[0].numpy()
    assert np.allclose(Phi.T @ Phi, N * N * np.eye(p), atol=1e-9)
    lam = np.sort(np.linalg.eigvalsh(A))
    h = 1.0 / (N + 1)
    for a, (k, l) in enumerate(F.prior_modes(N, p)):
        mu = 4 / h ** 2 * (np.sin(k * np.pi * h / 2) ** 2 + np.sin(l * np.pi * h / 2) ** 2)
        assert np.allclose(A @ Phi[:, a], mu * Phi[:, a], atol=1e-8 * N * mu)
    theta = np.sort([4 / h ** 2 * (np.sin(k * np.pi * h / 2) ** 2 + np.sin(l * np.pi * h / 2) ** 2)
                     for k, l in F.prior_modes(N, p)])
    assert np.allclose(theta, lam[:p], rtol=1e-12)


def test_loss_is_sum_of_squared_principal_angle_sines():
    g = np.random.default_rng(2)
    n, p = 40, 5
    Y = g.standard_normal((n, p))
    Xs, _ = np.linalg.qr(g.standard_normal((n, p)))
    ang = scipy.linalg.subspace_angles(Y, Xs)
    loss = F.subspace_loss(torch.tensor(Y[None]), torch.tensor(Xs[None]))[0].item()
    assert loss == pytest.approx(np.sum(np.sin(ang) ** 2), abs=1e-12)
    # invariant to a change of basis of Y, zero on the target subspace
    T = g.standard_normal((p, p))
    assert F.subspace_loss(torch.tensor((Y @ T)[None]), torch.tensor(Xs[None]))[0].item() == pytest.approx(loss, abs=1e-10)
    assert abs(F.subspace_loss(torch.tensor((Xs @ T)[None]), torch.tensor(Xs[None]))[0].item()) < 1e-12


def test_gradient_matches_central_differences():
    cfg = TINY
    g = np.random.default_rng(3)
    flat = _rand_params(cfg, 4)
    V = -20.0 * g.random((2, cfg.N * cfg.N))
    Xs = np.stack([np.linalg.qr(g.standard_normal((cfg.N * cfg.N, cfg.p)))[0] for _ in range(2)])
    loss, grad, _ = F.loss_and_grad(flat, V, Xs, cfg)
    idx = g.choice(flat.size, 40, replace=False)
    # include coordinates of every parameter group
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in F.param_shapes(cfg)])
    idx = np.unique(np.concatenate([idx, offs[:-1]]))
    h = 1e-6
    for i in idx:
        fp, fm = flat.copy(), flat.copy()
        fp[i] += h
        fm[i] -= h
        d = (F.loss_and_grad(fp, V, Xs, cfg)[0] - F.loss_and_grad(fm, V, Xs, cfg)[0]) / (2 * h)
        assert d == pytest.approx(grad[i], rel=1e-5, abs=1e-8), i


def test_adam_first_step_moves_each_weight_by_lr():
    # with bias correction the first update is lr * g / (|g| + eps), i.e. about lr * sign(g)
    flat = np.zeros(4)
    grad = np.array([3.0, -0.5, 1e-3, -2.0])
    m, v = np.zeros(4), np.zeros(4)
    F.adam_step(flat, grad, m, v, 1, lr=0.01)
    assert np.allclose(flat, -0.01 * np.sign(grad) * np.abs(grad) / (np.abs(grad) + 1e-8), atol=1e-15)


def test_forward_composes_the_layers_as_defined():
    """The whole forward pass recomputed from the architecture's definition with scipy's
    orthonormal DST-I (truncated to the m lowest modes) and erf, numpy products and the
    flat parameter layout: lift, L hidden layers gelu(K(U) + W U + b), output prior + K(U) +
    W U + b. Random parameters, several samples."""
    cfg = F.Config(N=10, m=4, w=3, L=2, p=3)
    flat = _rand_params(cfg, 21, scale=0.6)
    V = -20.0 * np.random.default_rng(22).random((2, cfg.N * cfg.N))
    N, m, w, p = cfg.N, cfg.m, cfg.w, cfg.p
    off = 0

    def take(*shape):
        nonlocal off
        size = int(np.prod(shape))
        out = flat[off:off + size].reshape(shape)
        off += size
        return out

    def K(U, R):
        Uh = scipy.fft.dstn(U, type=1, norm="ortho", axes=(2, 3))[:, :, :m, :m]
        full = np.zeros((U.shape[0], R.shape[0], N, N))
        full[:, :, :m, :m] = np.einsum("ocij,bcij->boij", R, Uh)
        return scipy.fft.idstn(full, type=1, norm="ortho", axes=(2, 3))

    def pw(U, W, b):
        return np.einsum("oc,bcij->boij", W, U) + b[None, :, None, None]

    def gelu(t):
        return 0.5 * t * (1.0 + scipy.special.erf(t / np.sqrt(2.0)))

    t = np.arange(1, N + 1) / (N + 1)
    In = np.stack([V.reshape(2, N, N) / 20.0, np.broadcast_to(t[None, :], (2, N, N)),
                   np.broadcast_to(t[:, None], (2, N, N))], axis=1)
    U = pw(In, take(w, 3), take(w))
    for _ in range(cfg.L):
        R, W, b = take(w, w, m, m), take(w, w), take(w)
        U = gelu(K(U, R) + pw(U, W, b))
    R, W, b = take(p, w, m, m), take(p, w), take(p)
    assert off == flat.size
    ref = F.prior(N, p).numpy()[None] + K(U, R) + pw(U, W, b)
    got = F.forward(torch.as_tensor(flat), torch.as_tensor(V), cfg).numpy()
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12)


def test_bf16_rounding_is_the_library_conversion():
    """round_bf16 against torch's float32 -> bfloat16 conversion (round to nearest even): random
    values over many binades, exact halfway cases of both parities, values one bit either side
    of a tie, a carry into the exponent, subnormals, signed zeros, infinities and the
    overflow to infinity."""
    g = np.random.default_rng(3)
    vals = [g.standard_normal(20000) * np.exp(g.uniform(-40, 40, 20000))]
    base = np.float32(1.0).view(np.uint32)
    ties = []
    for k in range(64):  # patterns kept | 0x8000 for even and odd kept parts, and neighbours
        kept = (base >> 16) + k
        for low in (0x7FFF, 0x8000, 0x8001):
            ties.append(np.uint32((kept << 16) | low))
    ties.append(np.uint32(0x3F7FFFFF))             # just below 1: carries into the exponent
    ties += [np.uint32(0x00008000), np.uint32(0x00018000), np.uint32(0x0000FFFF)]  # subnormal ties
    ties += [np.uint32(0x7F7FFFFF), np.uint32(0xFF7FFFFF)]  # largest finite: round to +-inf
    vals.append(np.array(ties, dtype=np.uint32).view(np.float32).astype(np.float64))
    vals.append(np.array([0.0, -0.0, np.inf, -np.inf, 1e-45, -1e-45]))
    x = np.concatenate(vals).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    got = F.round_bf16(x)
    assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))
    assert np.isnan(F.round_bf16(np.array([np.nan], np.float32))).all()
    # ties go to the even pattern: 1 + 2^-8 -> 1, 1 + 3 * 2^-8 -> 1 + 2^-6
    assert F.round_bf16(np.float32(1 + 2 ** -8)) == 1.0
    assert F.round_bf16(np.float32(1 + 3 * 2 ** -8)) == 1 + 2 ** -6
