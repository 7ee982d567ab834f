"""BF16-MFMA convolution kernels against the FP64 CNN oracle.

Single layers are compared with operands pre-rounded to BF16 on the oracle
side, so only the FP32-vs-FP64 accumulation differs (tight bound).  The full
network is compared twice: with the oracle rounding every convolution operand
to BF16 as the matrix cores do (relative 2e-3), and with the exact FP64
oracle, where four layers of BF16 operands cost up to ~2.5e-2 on the first
layer's weight gradient (bound 5e-2).
"""

import numpy as np
import pytest

from oracle import cnn as ocnn

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2607_24059_amd import cnn  # noqa: E402


bf16_round = ocnn.bf16_round


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


@pytest.mark.parametrize("cin,cout,relu", [(3, 32, True), (32, 32, True), (32, 3, False), (5, 20, False)])
def test_single_layer_forward(cin, cout, relu):
    rng = np.random.default_rng(cin * 100 + cout)
    B, H, W = 2, 6, 128
    x = rng.standard_normal((B, cin, H, W))
    w = rng.standard_normal((cout, cin, 3, 3)) * 0.3
    b = rng.standard_normal(cout)
    s = torch.cuda.current_stream()
    packed = torch.empty(cnn.lbm_conv_packed_bytes(cin, cout), dtype=torch.uint8, device="cuda")
    cnn.lbm_conv_pack(dev(w), cin, cout, 0, packed, s)
    y = torch.empty((B, cout, H, W), dtype=torch.float32, device="cuda")
    cnn.lbm_conv_forward(dev(x), B, cin, H, W, packed, cout, dev(b), None, 1 if relu else 0, y, s)
    ref = ocnn.conv(bf16_round(x), bf16_round(w), np.float32(b).astype(np.float64))
    if relu:
        ref = np.maximum(ref, 0)
    got = y.double().cpu().numpy()
    assert np.max(np.abs(got - ref)) <= 1e-5 * np.max(np.abs(ref)) + 1e-6


@pytest.mark.parametrize("cin,cout", [(3, 32), (32, 32), (32, 3)])
def test_single_layer_input_gradient_with_mask(cin, cout):
    """dX = conv(dY, W^T flipped), multiplied by (mask > 0)."""
    rng = np.random.default_rng(7 + cin)
    B, H, W = 2, 5, 64
    x = rng.standard_normal((B, cin, H, W))
    w = rng.standard_normal((cout, cin, 3, 3)) * 0.3
    dy = rng.standard_normal((B, cout, H, W))
    mask = rng.standard_normal((B, cin, H, W))
    s = torch.cuda.current_stream()
    packed = torch.empty(cnn.lbm_conv_packed_bytes(cin, cout), dtype=torch.uint8, device="cuda")
    cnn.lbm_conv_pack(dev(w), cin, cout, 1, packed, s)
    dx = torch.empty((B, cin, H, W), dtype=torch.float32, device="cuda")
    cnn.lbm_conv_forward(dev(dy), B, cout, H, W, packed, cin, None, dev(mask), 0, dx, s)
    ref, _, _ = ocnn.conv_backward(bf16_round(x), bf16_round(w), bf16_round(dy))
    ref = ref * (mask > 0)
    got = dx.double().cpu().numpy()
    assert np.max(np.abs(got - ref)) <= 1e-5 * np.max(np.abs(ref)) + 1e-6


@pytest.mark.parametrize("cin,cout,H", [(3, 32, 20), (32, 32, 17), (32, 3, 8)])
def test_single_layer_weight_gradient(cin, cout, H):
    rng = np.random.default_rng(11 + cout)
    B, W = 3, 128
    x = rng.standard_normal((B, cin, H, W))
    dy = rng.standard_normal((B, cout, H, W))
    s = torch.cuda.current_stream()
    dw = torch.empty((cout, cin, 3, 3), dtype=torch.float32, device="cuda")
    db = torch.empty(cout, dtype=torch.float32, device="cuda")
    nb = cnn.lbm_conv_wgrad_scratch_bytes(B, cin, cout, H, W)
    scratch = torch.empty(nb // 4, dtype=torch.float32, device="cuda")
    cnn.lbm_conv_wgrad(dev(x), dev(dy), B, cin, cout, H, W, dw, db, scratch, s)
    _, ref_w, _ = ocnn.conv_backward(bf16_round(x), np.zeros((cout, cin, 3, 3)), bf16_round(dy))
    ref_b = np.float32(dy).astype(np.float64).sum(axis=(0, 2, 3))
    assert np.max(np.abs(dw.double().cpu().numpy() - ref_w)) <= 1e-5 * np.max(np.abs(ref_w))
    assert np.max(np.abs(db.double().cpu().numpy() - ref_b)) <= 1e-5 * np.max(np.abs(ref_b))


def _net_case(seed=0, B=2, H=12, W=64):
    rng = np.random.default_rng(seed)
    params = ocnn.init_params(seed)
    params = [(w, 0.05 * rng.standard_normal(b.shape)) for w, b in params]
    x = rng.standard_normal((B, 3, H, W))
    t = rng.standard_normal((B, 3, H, W)) * 0.5
    return params, x, t


def test_network_forward_backward_matches_oracle():
    """Against the oracle with the GPU's operand rounding (every convolution
    operand rounded to BF16, FP64 arithmetic otherwise): only the FP32
    accumulation differs.  Against the exact FP64 oracle: the BF16 operand
    rounding through four layers, bounded at 5e-2 relative."""
    params, x, t = _net_case()
    net = cnn.Net(params)
    s = net.stream
    out = net.forward(dev(x))
    grad = torch.empty_like(out)
    loss_dev = cnn.mse(out, dev(t), grad, s)
    net.backward(grad)
    torch.cuda.synchronize()
    got_out = out.double().cpu().numpy()
    got = net.views(net.g.double().cpu().numpy())
    params32 = [(np.float32(w).astype(np.float64), np.float32(b).astype(np.float64)) for w, b in params]
    for rnd, tol in ((ocnn.bf16_round, 2e-3), (None, 5e-2)):
        kw = {} if rnd is None else {"rnd": rnd}
        ref_out, cache = ocnn.forward(params32, np.float32(x).astype(np.float64), **kw)
        ref_loss, dref = ocnn.mse(ref_out, t)
        grads, _ = ocnn.backward(params32, cache, dref, **kw)
        print(f"[cnn] rounding={'bf16' if rnd else 'none'}: out {rel(got_out, ref_out):.2e}, "
              + ", ".join(f"dW{li} {rel(gw, rw.ravel()):.2e}" for li, ((gw, _), (rw, _)) in enumerate(zip(got, grads))),
              flush=True)
        assert rel(got_out, ref_out) <= tol
        assert abs(loss_dev.item() - ref_loss) <= tol * ref_loss
        for li, ((gw, gb), (rw, rb)) in enumerate(zip(got, grads)):
            assert rel(gw, rw.ravel()) <= tol, li
            assert rel(gb, rb.ravel()) <= tol, li


def test_adam_matches_oracle():
    params, x, t = _net_case(1)
    net = cnn.Net(params)
    rng = np.random.default_rng(3)
    g = rng.standard_normal(net.n) * 1e-2
    opt = ocnn.Adam(params, lr=1e-3)
    ref_grads = []
    off = 0
    for w, b in params:
        gw = g[off:off + w.size].reshape(w.shape)
        off += w.size
        gb = g[off:off + b.size]
        off += b.size
        ref_grads.append((gw, gb))
    ref = params
    for _ in range(3):
        net.g.copy_(torch.tensor(g, dtype=torch.float32))
        net.adam_step(lr=1e-3)
        ref = opt.step(ref, ref_grads)
    got = net.host_params()
    for (w, b), (rw, rb) in zip(got, ref):
        assert np.max(np.abs(w - rw)) <= 1e-6 and np.max(np.abs(b - rb)) <= 1e-6


def test_training_reduces_loss():
    params, x, t = _net_case(2, B=4, H=8, W=64)
    net = cnn.Net(params)
    xd, td = dev(x), dev(t * 0.1)
    grad = torch.empty_like(td)
    losses = []
    for it in range(60):
        out = net.forward(xd)
        loss = cnn.mse(out, td, grad, net.stream)
        net.backward(grad)
        net.adam_step(lr=3e-3)
        if it % 10 == 0 or it == 59:
            losses.append(loss.item())
    assert losses[-1] < 0.5 * losses[0], losses


def test_channel_rms():
    rng = np.random.default_rng(4)
    x = rng.standard_normal((3, 5000)) * np.array([[1.0], [2.0], [0.5]])
    out = cnn.channel_rms(dev(x), 3, torch.cuda.current_stream())
    ref = np.sqrt(np.mean(np.float32(x).astype(np.float64) ** 2, axis=1))
    assert np.allclose(out.cpu().numpy(), ref, rtol=1e-12)


@pytest.mark.parametrize("h,w", [(16, 64), (48, 128), (64, 64)])
def test_fused_inference_equals_layer_by_layer(h, w):
    """lbm_net_infer (features + four layers in one launch, activations in LDS)
    gives the output of lbm_closure_features + four lbm_conv_forward calls bit
    for bit, and per-tile sums of that output."""
    from paper_2607_24059_amd import closure as cl
    rng = np.random.default_rng(h * 1000 + w)
    rho = 1 + 1e-3 * rng.standard_normal((h, w))
    q = 0.5 * rng.standard_normal((2, h, w))
    m = dev(np.concatenate([rho[None], q]))
    s_rho, s_u = 1e-3, 0.7
    net = cnn.Net(seed=h + w)
    s = torch.cuda.current_stream()
    x = torch.empty((1, 3, h, w), dtype=torch.float32, device="cuda")
    cl.lbm_closure_features(m, 2, h * w, 1.0, s_rho, s_u, x, s)
    ref = net.forward(x)[0].clone()
    y = torch.empty((3, h, w), dtype=torch.float32, device="cuda")
    part = torch.empty(cnn.lbm_net_partials_bytes(h, w) // 8, dtype=torch.float64, device="cuda")
    cnn.lbm_net_infer(m, h, w, 1.0, s_rho, s_u, net, y, part, s)
    torch.cuda.synchronize()
    assert torch.equal(y, ref)
    yh = y.double().cpu().numpy()
    sums = yh.reshape(3, h // 16, 16, w // 16, 16).sum(axis=(2, 4))  # [3][ty][tx]
    got = part.cpu().numpy().reshape(-1, 4)
    assert np.allclose(got[:, :3], sums.reshape(3, -1).T, rtol=1e-12, atol=1e-12 * np.abs(yh).sum())
    assert np.all(got[:, 3] == 0)


def test_fused_inference_rejects_ragged_shapes():
    net = cnn.Net(seed=0)
    m = torch.ones((3, 40, 64), dtype=torch.float32, device="cuda")
    y = torch.empty_like(m)
    part = torch.empty(64, dtype=torch.float64, device="cuda")
    assert cnn.lbm_net_partials_bytes(40, 64) == 0
    with pytest.raises(cnn.LbmError):
        cnn.lbm_net_infer(m, 40, 64, 1.0, 1.0, 1.0, net, y, part, torch.cuda.current_stream())
