"""GPU scorer kernels against the CPU reference (fp64 with bf16 rounding at
the same storage points): forward activations and outputs, gradients within
2^-7 of the largest gradient entry (plus 1e-6), and one Adam step."""
import numpy as np
import pytest

from oracle import mlp_ref

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2601_21552_amd import api
    return torch, api, api.Context(0)


def _ulp(v):
    """Spacing of bf16 values at |v| (0 for 0)."""
    a = np.abs(np.asarray(v, np.float64))
    e = np.floor(np.log2(np.where(a > 0, a, 1.0)))
    return np.where(a > 0, 2.0 ** (e - 7), 0.0)


def _case(seed, B):
    rng = np.random.Generator(np.random.PCG64(seed))
    p = mlp_ref.init_params(rng)
    p["b1"] = (rng.standard_normal(128) * 0.1).astype(np.float32)
    p["b2"] = (rng.standard_normal(128) * 0.1).astype(np.float32)
    p["b3"] = np.array([0.3], np.float32)
    X = rng.standard_normal((B, 16)).astype(np.float32)
    t = rng.standard_normal(B).astype(np.float32)
    return p, X, t


@pytest.mark.parametrize("B", [1, 16, 37, 100, 513, 1024])
def test_forward_and_backward_match_reference(env, B):
    torch, api, ctx = env
    p, X, t = _case(40 + B, B)
    mlp = api.Mlp(ctx, api.mlp_flatten(p))
    x = torch.tensor(X, device="cuda").to(torch.bfloat16)
    y, a1, a2 = mlp.forward(x)
    y_ref, c = mlp_ref.forward(p, X)
    torch.cuda.synchronize()
    A1 = a1.float().cpu().numpy()
    A2 = a2.float().cpu().numpy()
    # Layer 1: within one bf16 ulp of the reference (fp32 vs fp64 sums may
    # round either way), plus accumulation noise next to the ReLU threshold.
    # Layer 2 inherits layer 1's one-ulp flips through W2: its bound adds
    # sum_k ulp(A1[k]) |W2[k][j]|, and y adds sum_j |dA2[j]| |w3[j]|.
    W2 = mlp_ref.bf16_round(p["W2"])
    w3 = mlp_ref.bf16_round(p["w3"])
    noise = 2.0 ** -16
    tol1 = _ulp(c["A1"]) + noise * np.max(np.abs(c["A1"]))
    assert np.all(np.abs(A1 - c["A1"]) <= tol1), np.max(np.abs(A1 - c["A1"]) / tol1)
    tol2 = _ulp(c["A2"]) + tol1 @ np.abs(W2) + noise * np.max(np.abs(c["A2"]))
    assert np.all(np.abs(A2 - c["A2"]) <= tol2), np.max(np.abs(A2 - c["A2"]) / tol2)
    yv = y.cpu().numpy()
    toly = tol2 @ np.abs(w3) + 2.0 ** -20 * (np.abs(y_ref) + 1)
    assert np.all(np.abs(yv - y_ref) <= toly), np.max(np.abs(yv - y_ref) / toly)
    g_ref, _ = mlp_ref.backward(p, X, t)
    grad = mlp.backward(x, a1, a2, y, torch.tensor(t, device="cuda"))
    torch.cuda.synchronize()
    g = api.mlp_unflatten(grad.cpu().numpy())
    for k in g_ref:
        bound = 2.0 ** -7 * np.max(np.abs(g_ref[k])) + 1e-6
        assert np.max(np.abs(g[k] - g_ref[k])) <= bound, (k, np.max(np.abs(g[k] - g_ref[k])), bound)


def test_adam_step_matches_reference(env):
    torch, api, ctx = env
    p, X, t = _case(7, 64)
    mlp = api.Mlp(ctx, api.mlp_flatten(p))
    x = torch.tensor(X, device="cuda").to(torch.bfloat16)
    y, a1, a2 = mlp.forward(x)
    grad = mlp.backward(x, a1, a2, y, torch.tensor(t, device="cuda"))
    g = api.mlp_unflatten(grad.cpu().numpy())
    mlp.adam(lr=1e-2)
    torch.cuda.synchronize()
    ref = {k: v.copy() for k, v in p.items()}
    m = {k: np.zeros_like(v, np.float64) for k, v in p.items()}
    v = {k: np.zeros_like(x_, np.float64) for k, x_ in p.items()}
    mlp_ref.adam_step(ref, {k: g[k].astype(np.float64) for k in g}, m, v, 1, lr=1e-2)
    got = api.mlp_unflatten(mlp.params())
    for k in ref:
        assert np.allclose(got[k], ref[k], rtol=1e-5, atol=1e-6), k


def test_training_reduces_loss(env):
    torch, api, ctx = env
    rng = np.random.Generator(np.random.PCG64(9))
    p = mlp_ref.init_params(rng)
    X = rng.standard_normal((512, 16)).astype(np.float32)
    t = (np.tanh(X[:, 0]) - 0.5 * X[:, 1] * X[:, 2]).astype(np.float32)
    mlp = api.Mlp(ctx, api.mlp_flatten(p))
    x = torch.tensor(X, device="cuda").to(torch.bfloat16)
    tt = torch.tensor(t, device="cuda")
    losses = []
    for _ in range(150):
        y, a1, a2 = mlp.forward(x)
        losses.append(float(((y - tt) ** 2).mean()))
        mlp.backward(x, a1, a2, y, tt)
        mlp.adam(lr=2e-3)
    assert losses[-1] < 0.3 * losses[0], losses[::30]
