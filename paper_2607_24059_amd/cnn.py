"""ctypes binding of the convolution kernels (include/lbm_cnn.h) and a small
network driver built on them.

Every arithmetic step runs in liblbm.so; this module marshals arguments and
sequences the calls (forward, backward, Adam) of the four-layer correction
network: 3x3 periodic convolutions 3 -> 32 -> 32 -> 32 -> 3 with ReLU after
the first three.
"""

from __future__ import annotations

import ctypes as C

import numpy as np

from .lbm import LbmError, _ok, lib

LAYERS = ((3, 32), (32, 32), (32, 32), (32, 3))
LBM_CONV_RELU = 0x1

SIGNATURES = {
    "lbm_conv_packed_bytes": (C.c_size_t, [C.c_int32, C.c_int32]),
    "lbm_conv_pack": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p]),
    "lbm_conv_forward": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                   C.c_int32, C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p]),
    "lbm_conv_wgrad_scratch_bytes": (C.c_size_t, [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    "lbm_conv_wgrad": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                 C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "lbm_reduce_scratch_bytes": (C.c_size_t, [C.c_int64]),
    "lbm_mse": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "lbm_adam": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_float, C.c_float,
                           C.c_float, C.c_float, C.c_int32, C.c_void_p]),
    "lbm_channel_rms": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]),
    "lbm_net_partials_bytes": (C.c_size_t, [C.c_int32, C.c_int32]),
    "lbm_net_infer": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_double, C.c_float, C.c_float,
                                C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_void_p, C.c_void_p,
                                C.c_void_p]),
}

_bound = False


def clib():
    global _bound
    L = lib()
    if not _bound:
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _bound = True
    return L


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _s(stream):
    return C.c_void_p(stream.cuda_stream)


def lbm_conv_packed_bytes(cin, cout):
    return int(clib().lbm_conv_packed_bytes(cin, cout))


def lbm_conv_pack(w, cin, cout, transpose, packed, stream):
    _ok(clib().lbm_conv_pack(_p(w), cin, cout, int(transpose), _p(packed), _s(stream)), "lbm_conv_pack")


def lbm_conv_forward(x, batch, cin, h, w, packed, cout, bias, mask, flags, y, stream):
    _ok(clib().lbm_conv_forward(_p(x), batch, cin, h, w, _p(packed), cout, _p(bias), _p(mask), flags, _p(y),
                                _s(stream)), "lbm_conv_forward")


def lbm_conv_wgrad_scratch_bytes(batch, cin, cout, h, w):
    return int(clib().lbm_conv_wgrad_scratch_bytes(batch, cin, cout, h, w))


def lbm_conv_wgrad(x, dy, batch, cin, cout, h, w, dw, db, scratch, stream):
    _ok(clib().lbm_conv_wgrad(_p(x), _p(dy), batch, cin, cout, h, w, _p(dw), _p(db), _p(scratch), _s(stream)),
        "lbm_conv_wgrad")


def lbm_reduce_scratch_bytes(n):
    return int(clib().lbm_reduce_scratch_bytes(n))


def lbm_mse(out, target, n, grad, loss_dev, scratch, stream):
    _ok(clib().lbm_mse(_p(out), _p(target), n, _p(grad), _p(loss_dev), _p(scratch), _s(stream)), "lbm_mse")


def lbm_net_partials_bytes(h, w):
    return int(clib().lbm_net_partials_bytes(h, w))


def lbm_net_infer(moments, h, w, rho_ref, s_rho, s_u, net, y, partials, stream):
    packed, bias = net.layer_pointers()
    _ok(clib().lbm_net_infer(_p(moments), h, w, rho_ref, s_rho, s_u, packed, bias, _p(y), _p(partials),
                             _s(stream)), "lbm_net_infer")


def lbm_adam(p, g, m, v, n, lr, b1, b2, eps, t, stream):
    _ok(clib().lbm_adam(_p(p), _p(g), _p(m), _p(v), n, lr, b1, b2, eps, t, _s(stream)), "lbm_adam")


def lbm_channel_rms(x, channels, n, out_dev, scratch, stream):
    _ok(clib().lbm_channel_rms(_p(x), channels, n, _p(out_dev), _p(scratch), _s(stream)), "lbm_channel_rms")


class Net:
    """Parameters (flat FP32: W1 b1 W2 b2 W3 b3 W4 b4), packed BF16 operands,
    activations and gradients of the correction network on one device."""

    def __init__(self, params=None, seed: int = 0, device="cuda"):
        import torch
        self.torch = torch
        self.layers = LAYERS
        sizes = []
        for cin, cout in LAYERS:
            sizes += [cout * cin * 9, cout]
        self.sizes = sizes
        self.n = sum(sizes)
        if params is None:
            rng = np.random.default_rng(seed)
            flat = []
            for cin, cout in LAYERS:
                bound = np.sqrt(6.0 / (cin * 9))
                flat += [rng.uniform(-bound, bound, cout * cin * 9), np.zeros(cout)]
            host = np.concatenate(flat)
        else:
            host = np.concatenate([np.concatenate([np.asarray(w, dtype=np.float64).ravel(),
                                                   np.asarray(b, dtype=np.float64).ravel()]) for w, b in params])
        assert host.size == self.n
        self.p = torch.tensor(host, dtype=torch.float32, device=device)
        self.g = torch.zeros_like(self.p)
        self.m = torch.zeros_like(self.p)
        self.v = torch.zeros_like(self.p)
        self.t = 0
        self.packed = [torch.empty(lbm_conv_packed_bytes(ci, co), dtype=torch.uint8, device=device)
                       for ci, co in LAYERS]
        self.packed_t = [torch.empty(lbm_conv_packed_bytes(ci, co), dtype=torch.uint8, device=device)
                         for ci, co in LAYERS]
        self._acts = {}
        self.repack()

    @property
    def stream(self):
        """Every launch goes to torch's current stream (so a caller can capture it)."""
        return self.torch.cuda.current_stream()

    def views(self, flat):
        out, off = [], 0
        for li, (cin, cout) in enumerate(LAYERS):
            nw, nb = cout * cin * 9, cout
            out.append((flat[off:off + nw], flat[off + nw:off + nw + nb]))
            off += nw + nb
        return out

    def repack(self):
        for li, (cin, cout) in enumerate(LAYERS):
            w, _ = self.views(self.p)[li]
            lbm_conv_pack(w, cin, cout, 0, self.packed[li], self.stream)
            lbm_conv_pack(w, cin, cout, 1, self.packed_t[li], self.stream)

    def layer_pointers(self):
        """Host arrays of the four layers' forward-packed operands and biases (device pointers)."""
        packed = (C.c_void_p * 4)(*[t.data_ptr() for t in self.packed])
        bias = (C.c_void_p * 4)(*[b.data_ptr() for _, b in self.views(self.p)])
        return packed, bias

    def host_params(self):
        flat = self.p.double().cpu().numpy()
        out = []
        for (w, b), (cin, cout) in zip(self.views(flat), LAYERS):
            out.append((w.reshape(cout, cin, 3, 3).copy(), b.copy()))
        return out

    def _buf(self, key, shape):
        t = self._acts.get(key)
        if t is None or tuple(t.shape) != tuple(shape):
            t = self.torch.empty(shape, dtype=self.torch.float32, device=self.p.device)
            self._acts[key] = t
        return t

    def forward(self, x):
        """x: [B, 3, H, W] FP32 device tensor -> output [B, 3, H, W]; keeps activations."""
        B, _, H, W = x.shape
        a = x
        self._x = x
        self._a = []
        for li, (cin, cout) in enumerate(LAYERS):
            last = li == len(LAYERS) - 1
            y = self._buf(("a", li), (B, cout, H, W))
            _, bias = self.views(self.p)[li]
            lbm_conv_forward(a, B, cin, H, W, self.packed[li], cout, bias, None,
                             0 if last else LBM_CONV_RELU, y, self.stream)
            self._a.append(y)
            a = y
        return a

    def backward(self, dout):
        """Gradients into self.g from dL/doutput (after forward on the same input)."""
        B, _, H, W = dout.shape
        gv = self.views(self.g)
        d = dout
        for li in range(len(LAYERS) - 1, -1, -1):
            cin, cout = LAYERS[li]
            a_in = self._x if li == 0 else self._a[li - 1]
            nbytes = lbm_conv_wgrad_scratch_bytes(B, cin, cout, H, W)
            scratch = self._buf(("ws", li), (nbytes // 4,))
            lbm_conv_wgrad(a_in, d, B, cin, cout, H, W, gv[li][0], gv[li][1], scratch, self.stream)
            if li > 0:
                dn = self._buf(("d", li), (B, cin, H, W))
                # dX = conv(dY, W^T flipped); times the ReLU mask of the layer below
                lbm_conv_forward(d, B, cout, H, W, self.packed_t[li], cin, None, a_in, 0, dn, self.stream)
                d = dn

    def adam_step(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.t += 1
        lbm_adam(self.p, self.g, self.m, self.v, self.n, lr, b1, b2, eps, self.t, self.stream)
        self.repack()


def mse(out, target, grad, stream, scratch=None, loss_dev=None):
    import torch
    n = out.numel()
    if scratch is None:
        scratch = torch.empty(lbm_reduce_scratch_bytes(n) // 4, dtype=torch.float32, device=out.device)
    if loss_dev is None:
        loss_dev = torch.empty(1, dtype=torch.float64, device=out.device)
    lbm_mse(out, target, n, grad, loss_dev, scratch, stream)
    return loss_dev


def channel_rms(x, channels, stream):
    import torch
    n = x.numel() // channels
    scratch = torch.empty(lbm_reduce_scratch_bytes(n) // 4, dtype=torch.float32, device=x.device)
    out = torch.empty(channels, dtype=torch.float64, device=x.device)
    lbm_channel_rms(x, channels, n, out, scratch, stream)
    return out


__all__ = ["Net", "LAYERS", "LbmError", "mse", "channel_rms"]
