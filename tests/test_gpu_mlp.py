"""GPU parity of the surrogate MLP kernels against the FP64 oracle:
forward (fp32) and backward gradients within 1e-4 relative, one Adam step,
bf16 inference against the fp32 forward, and a short training run that
lowers the loss."""
import numpy as np
import pytest

from oracle import mlp as L
from tests.gpu_common import lib

pytestmark = pytest.mark.gpu


def _dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    return t.to("cuda", dtype or torch.float32)


@pytest.mark.parametrize("B", [1, 77, 512])
def test_forward_backward_vs_fp64(gpu, B):
    import torch
    P = lib()
    rng = np.random.default_rng(B)
    p = L.init(2)
    x = rng.uniform(-1, 1, size=(B, 12))
    dy = rng.normal(size=B)
    y_o, cache = L.forward(p, x)
    g_o = L.backward(p, cache, dy)
    pt, xt, dyt = _dev(p), _dev(x), _dev(dy)
    y = torch.empty(B, device="cuda")
    g = torch.empty(P.mlp_param_count(), device="cuda")
    ws = torch.empty(P.mlp_workspace_bytes(B), dtype=torch.uint8, device="cuda")
    P.mlp_forward(pt, xt, y, ws)
    P.mlp_backward(pt, xt, dyt, g, ws)
    torch.cuda.synchronize()
    yg, gg = y.cpu().numpy().astype(np.float64), g.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(yg - y_o)) <= 1e-5 * max(1.0, np.max(np.abs(y_o)))
    rel = np.linalg.norm(gg - g_o) / np.linalg.norm(g_o)
    print("grad rel err", rel)
    assert rel < 1e-4
    # per-layer check, so a wrong block cannot hide in the global norm
    o = 0
    for name, s in L.SHAPES:
        k = int(np.prod(s))
        blk_o, blk_g = g_o[o:o + k], gg[o:o + k]
        assert np.linalg.norm(blk_g - blk_o) <= 1e-4 * np.linalg.norm(blk_o) + 1e-6 * np.linalg.norm(g_o), name
        o += k


def test_adam_step_vs_oracle(gpu):
    import torch
    P = lib()
    rng = np.random.default_rng(9)
    n = P.mlp_param_count()
    p, g = rng.normal(size=n), rng.normal(size=n)
    m, v = rng.normal(size=n) * 0.1, rng.random(n) * 0.1
    q_o, m_o, v_o = L.adam(p, g, m, v, 5, lr=1e-3)
    pt, gt, mt, vt = _dev(p), _dev(g), _dev(m), _dev(v)
    P.mlp_adam_step(pt, gt, mt, vt, 5, lr=1e-3)
    torch.cuda.synchronize()
    assert np.allclose(pt.cpu().numpy(), q_o, rtol=1e-5, atol=1e-6)
    assert np.allclose(mt.cpu().numpy(), m_o, rtol=1e-5, atol=1e-7)


def test_bf16_inference_close_to_fp32(gpu):
    import torch
    P = lib()
    rng = np.random.default_rng(5)
    p = L.init(4)
    x = rng.uniform(-1, 1, size=(1000, 12))
    y_o, _ = L.forward(p, x)
    pt = _dev(p)
    packed = torch.empty(P.mlp_param_count(), dtype=torch.bfloat16, device="cuda")
    P.mlp_pack_bf16(pt, packed)
    y = torch.empty(1000, device="cuda")
    P.mlp_infer_bf16(packed, _dev(x), y)
    torch.cuda.synchronize()
    err = np.abs(y.cpu().numpy() - y_o)
    print("bf16 max abs err", err.max(), "scale", np.abs(y_o).max())
    assert err.max() < 3e-2 * max(1.0, np.abs(y_o).max())


def test_training_lowers_loss(gpu):
    import torch
    P = lib()
    rng = np.random.default_rng(6)
    x = rng.uniform(-1, 1, size=(512, 12))
    t = np.sin(x @ rng.normal(size=12)) + 0.5 * x[:, 0] ** 2
    pt = _dev(L.init(7))
    m = torch.zeros_like(pt)
    v = torch.zeros_like(pt)
    xt, tt = _dev(x), _dev(t)
    y = torch.empty(512, device="cuda")
    g = torch.empty_like(pt)
    ws = torch.empty(P.mlp_workspace_bytes(512), dtype=torch.uint8, device="cuda")
    losses = []
    for step in range(1, 301):
        P.mlp_forward(pt, xt, y, ws)
        dy = 2.0 * (y - tt) / 512
        losses.append(float(((y - tt) ** 2).mean()))
        P.mlp_backward(pt, xt, dy, g, ws)
        P.mlp_adam_step(pt, g, m, v, step, lr=1e-3)
    torch.cuda.synchronize()
    print("loss", losses[0], losses[-1])
    assert losses[-1] < 0.1 * losses[0]
