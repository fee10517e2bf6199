"""Float64 CPU reference of the sine-basis neural operator used for learned warm starts.

TEST INFRASTRUCTURE ONLY. Imported by tests and by the package's smoke check, by nothing
else; it shares no code with the device network. Plain PyTorch CPU operations in float64,
with torch.autograd giving the exact derivative of the forward pass as written here.

The network maps a potential V on the N x N interior grid of the unit square (the
Schroedinger operators of Sec. 6-style test problems, H = -Laplacian + V) to a block Y of
p columns whose span is meant to approximate the invariant subspace of H's p smallest
eigenvalues. The method's convergence is governed by the angles between the start block and
that subspace (the rates of Sec. 4 apply from the starting angle on), so a start block with
small angles saves iterations; the subspace iteration itself still runs to the tolerance.

Architecture (widths w, sine modes m, L hidden layers, p outputs):
  inputs  In = [V / 20, x, y]                        (3 channels; x varies along a grid row)
  lift    U_0 = W_lift In + b_lift                   (pointwise, 3 -> w)
  layer l U_{l+1} = gelu(K_l(U_l) + W_l U_l + b_l)   (l = 0 .. L-1; w -> w)
  output  Y = Phi + K_out(U_L) + W_out U_L + b_out   (w -> p, no activation)
  K(U)[o] = S^T ( sum_c R[o, c] * (S U[c] S^T) ) S   (elementwise product over the m x m
            sine coefficients), S[k, i] = sqrt(2/(N+1)) sin(pi (k+1)(i+1)/(N+1)), k < m:
            the first m rows of the orthonormal type-I sine transform.
  gelu(t) = t Phi_n(t) with Phi_n the standard normal distribution function.
  Phi: fixed prior, column a = sqrt(n) times the a-th lowest Dirichlet mode of the grid
       Laplacian, phi_{k,l}[row r][col c] = s_l(r) s_k(c) with s_k(i) = sqrt(2/(N+1))
       sin(pi k (i+1)/(N+1)), ordered by k^2 + l^2, then k. These are the exact eigenvectors
       of the 5-point Laplacian, i.e. the answer for V = 0, so the network learns the
       correction that the potential makes; with a zero output layer it returns Phi.
Loss of one sample, with Y read as an n x p matrix (n = N^2) and X* the target orthonormal
basis: loss = p - Tr(G^-1 B^T B), G = Y^T Y, B = X*^T Y, i.e. the squared Frobenius norm of
the projection of X* off span(Y) = the sum of squared sines of the principal angles. A batch
loss is the mean over samples.

Flat parameter layout (one vector, in this order): W_lift (w x 3, [c][a]), b_lift (w); for
each hidden layer R (w x w x m x m, [o][c][k1][k2]), W (w x w, [o][c]), b (w); then R_out
(p x w x m x m), W_out (p x w), b_out (p).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch


@dataclass(frozen=True)
class Config:
    N: int = 256   # grid side
    m: int = 24    # sine modes per direction
    w: int = 20    # width
    L: int = 4     # hidden spectral layers
    p: int = 32    # output channels (block size)


def param_shapes(cfg: Config):
    w, m, p = cfg.w, cfg.m, cfg.p
    shapes = [("W_lift", (w, 3)), ("b_lift", (w,))]
    for l in range(cfg.L):
        shapes += [(f"R{l}", (w, w, m, m)), (f"W{l}", (w, w)), (f"b{l}", (w,))]
    shapes += [("R_out", (p, w, m, m)), ("W_out", (p, w)), ("b_out", (p,))]
    return shapes


def param_count(cfg: Config) -> int:
    return int(sum(np.prod(s) for _, s in param_shapes(cfg)))


def unflatten(flat: torch.Tensor, cfg: Config) -> dict:
    out, off = {}, 0
    for name, shape in param_shapes(cfg):
        size = int(np.prod(shape))
        out[name] = flat[off:off + size].reshape(shape)
        off += size
    return out


def sine_basis(N: int, m: int) -> torch.Tensor:
    """First m rows of the orthonormal type-I discrete sine transform of length N."""
    k = torch.arange(1, m + 1, dtype=torch.float64)[:, None]
    i = torch.arange(1, N + 1, dtype=torch.float64)[None, :]
    return np.sqrt(2.0 / (N + 1)) * torch.sin(np.pi * k * i / (N + 1))


def features(V: torch.Tensor, N: int) -> torch.Tensor:
    """V: (B, N*N) potential at the grid nodes in row-major order -> (B, 3, N, N)."""
    B = V.shape[0]
    t = torch.arange(1, N + 1, dtype=torch.float64) / (N + 1)
    x = t[None, :].expand(N, N)   # varies along a row
    y = t[:, None].expand(N, N)   # varies down the rows
    return torch.stack([V.reshape(B, N, N) / 20.0, x.expand(B, N, N), y.expand(B, N, N)], dim=1)


def spectral(U: torch.Tensor, R: torch.Tensor, S: torch.Tensor) -> torch.Tensor:
    """K(U) for U (B, C, N, N), R (O, C, m, m)."""
    Uh = S @ U @ S.T                                   # (B, C, m, m)
    Vh = torch.einsum("ocij,bcij->boij", R, Uh)        # mode-wise channel mixing
    return S.T @ Vh @ S                                # (B, O, N, N)


def pointwise(U: torch.Tensor, W: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    return torch.einsum("oc,bcij->boij", W, U) + b[None, :, None, None]


def gelu(t: torch.Tensor) -> torch.Tensor:
    return 0.5 * t * (1.0 + torch.erf(t / np.sqrt(2.0)))


def prior_modes(N: int, p: int):
    """(k, l) of the p lowest Dirichlet modes, ordered by k^2 + l^2, then k."""
    K = int(np.ceil(np.sqrt(2 * p))) + 2
    return sorted(((k, l) for k in range(1, K + 1) for l in range(1, K + 1)), key=lambda t: (t[0] ** 2 + t[1] ** 2, t[0]))[:p]


def prior(N: int, p: int) -> torch.Tensor:
    """Phi as (p, N, N): sqrt(n) times the unit-norm sampled modes."""
    i = torch.arange(1, N + 1, dtype=torch.float64)
    s = lambda k: np.sqrt(2.0 / (N + 1)) * torch.sin(np.pi * k * i / (N + 1))
    return torch.stack([N * torch.outer(s(l), s(k)) for k, l in prior_modes(N, p)])


def forward(flat: torch.Tensor, V: torch.Tensor, cfg: Config) -> torch.Tensor:
    """Returns Y as (B, p, N, N): channel a of sample b is column a of its n x p block."""
    P = unflatten(flat, cfg)
    S = sine_basis(cfg.N, cfg.m)
    U = pointwise(features(V, cfg.N), P["W_lift"], P["b_lift"])
    for l in range(cfg.L):
        U = gelu(spectral(U, P[f"R{l}"], S) + pointwise(U, P[f"W{l}"], P[f"b{l}"]))
    return prior(cfg.N, cfg.p)[None] + spectral(U, P["R_out"], S) + pointwise(U, P["W_out"], P["b_out"])


def as_blocks(Y: torch.Tensor) -> torch.Tensor:
    """(B, p, N, N) -> (B, n, p)."""
    B, p = Y.shape[:2]
    return Y.reshape(B, p, -1).transpose(1, 2)


def subspace_loss(Yb: torch.Tensor, Xs: torch.Tensor) -> torch.Tensor:
    """Per-sample p - Tr(G^-1 B^T B), Yb and Xs (B, n, p) with orthonormal Xs columns."""
    G = Yb.transpose(1, 2) @ Yb
    Bm = Xs.transpose(1, 2) @ Yb
    M = Bm.transpose(1, 2) @ Bm
    return Yb.shape[2] - torch.diagonal(torch.linalg.solve(G, M), dim1=1, dim2=2).sum(-1)


def loss_and_grad(flat: np.ndarray, V: np.ndarray, Xs: np.ndarray, cfg: Config):
    """Mean loss over the batch and its gradient with respect to the flat parameters.
    V: (B, n); Xs: (B, n, p) orthonormal targets."""
    f = torch.tensor(np.asarray(flat, dtype=np.float64), requires_grad=True)
    Y = forward(f, torch.as_tensor(np.asarray(V, dtype=np.float64)), cfg)
    per = subspace_loss(as_blocks(Y), torch.as_tensor(np.asarray(Xs, dtype=np.float64)))
    loss = per.mean()
    loss.backward()
    return float(loss.detach()), f.grad.numpy().copy(), per.detach().numpy().copy()


def predict(flat: np.ndarray, V: np.ndarray, cfg: Config) -> np.ndarray:
    """Y as (B, n, p) float64."""
    with torch.no_grad():
        Y = forward(torch.as_tensor(np.asarray(flat, dtype=np.float64)), torch.as_tensor(np.asarray(V, dtype=np.float64)),
                    cfg)
    return as_blocks(Y).numpy().copy()


def adam_step(flat, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015, Algorithm 1), t = step number from 1; in place."""
    m[:] = beta1 * m + (1.0 - beta1) * grad
    v[:] = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    flat[:] = flat - lr * mh / (np.sqrt(vh) + eps)


def round_bf16(x) -> np.ndarray:
    """bfloat16 value of each float32 entry of x, as float64. bfloat16 keeps binary32's sign
    and 8-bit exponent and the top 7 fraction bits: the 16 low bits of the binary32 pattern are
    rounded away to nearest, ties to the even pattern (a carry may step the exponent, and
    the largest finite values round to infinity); NaN stays NaN. The weights of the network in
    its bfloat16 mode are these values of the float32 parameters."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    kept = u >> 16
    rest = u & 0xFFFF
    up = (rest > 0x8000) | ((rest == 0x8000) & (kept & 1 == 1))
    bits = ((kept + up) << 16).astype(np.uint32)
    out = bits.view(np.float32).astype(np.float64)
    out[np.isnan(a)] = np.nan
    return out
