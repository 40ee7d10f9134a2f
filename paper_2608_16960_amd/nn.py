"""ctypes binding of libtspnn.so (include/tspnn.h) and the layers built on it.

- residual, dot, axpy, scale: the per-object vector steps of the solvers;
- tv(rho, eps): smoothed anisotropic total variation and its gradient;
- TV: torch.autograd.Function around it (for lambda * TV(rho) in a loss);
- Adam: optimiser state in device memory, one fused update kernel per step;
- CNN: the 6-layer 3-D CNN on the (r, e, a) grid (1 -> 32 -> 32 -> 32 -> 32 ->
  32 -> 1, ReLU between, circular padding in azimuth, residual output),
  forward and backward entirely in the HIP kernels (BF16 MFMA with FP32
  accumulation for the 32 -> 32 layers).

Argument marshalling only: every computation runs in the native library, and
importing this module fails when libtspnn.so is missing.
"""
import ctypes
import os

import numpy as np
import torch

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libtspnn.so")

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_f = ctypes.c_float
_st = ctypes.c_int

SIGNATURES = {
    "tspnn_tv_workspace": (ctypes.c_size_t, [_i32, _i64]),
    "tspnn_tv": (_st, [_vp, _i32, _i32, _i32, _i32, _f, _vp, _vp, _vp, _vp]),
    "tspnn_adam": (_st, [_vp, _vp, _vp, _vp, _i64, _f, _f, _f, _f, _f, _i32, _vp, _vp]),
    "tspnn_conv_workspace": (ctypes.c_size_t, [_i32, _i32, _i32, _i32]),
    "tspnn_conv_in_fwd": (_st, [_vp, _i32, _i32, _i32, _i32, _vp, _vp, _vp, _vp]),
    "tspnn_conv_fwd": (_st, [_vp, _i32, _i32, _i32, _i32, _vp, _vp, _vp, _vp]),
    "tspnn_conv_out_fwd": (_st, [_vp, _i32, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp]),
    "tspnn_conv_bwd_data": (_st, [_vp, _i32, _i32, _i32, _i32, _vp, _vp, _vp, _vp]),
    "tspnn_conv_bwd_weight": (_st, [_vp, _vp, _i32, _i32, _i32, _i32, _vp, _vp, _vp, _vp]),
    "tspnn_conv_in_bwd_weight": (_st, [_vp, _vp, _i32, _i32, _i32, _i32, _vp, _vp, _vp, _vp]),
    "tspnn_conv_out_bwd": (_st, [_vp, _vp, _i32, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp,
                                 _vp]),
    "tspnn_conv_flip_weights": (_st, [_vp, _vp, _vp]),
    "tspnn_to_bf16": (_st, [_vp, _vp, _i64, _vp]),
    "tspnn_from_bf16": (_st, [_vp, _vp, _i64, _vp]),
    "tspnn_vec_workspace": (ctypes.c_size_t, [_i32, _i64]),
    "tspnn_residual": (_st, [_vp, _vp, _i32, _i64, _vp, _vp, _vp, _vp, _vp]),
    "tspnn_dot": (_st, [_vp, _vp, _i32, _i64, _vp, _vp, _vp]),
    "tspnn_axpy": (_st, [_vp, _vp, _f, _i32, _i64, _vp, _vp]),
    "tspnn_scale": (_st, [_vp, _f, _i64, _vp, _vp]),
    "tspnn_stream_copy": (_st, [_vp, _vp, _i64, _i32, _vp]),
    "tspnn_stream_read": (_st, [_vp, _i64, _i32, _vp, _vp]),
    "tspnn_last_error": (ctypes.c_char_p, []),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2608_16960_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


class TspnnError(RuntimeError):
    pass


def check(status):
    if status != 0:
        raise TspnnError(f"tspnn status {status}: {lib.tspnn_last_error().decode(errors='replace')}")


def _p(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _s():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _req(t, dtype, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype:
        raise ValueError(f"{name} must be a CUDA {dtype} tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


# ------------------------------------------------------------------ bf16

def to_bf16(x):
    """float32 -> bfloat16 (round to nearest even) by the library kernel."""
    x = _req(x.contiguous(), torch.float32, "x")
    y = torch.empty(x.shape, dtype=torch.bfloat16, device=x.device)
    check(lib.tspnn_to_bf16(_p(x), _p(y), x.numel(), _s()))
    return y


def from_bf16(x):
    x = _req(x.contiguous(), torch.bfloat16, "x")
    y = torch.empty(x.shape, dtype=torch.float32, device=x.device)
    check(lib.tspnn_from_bf16(_p(x), _p(y), x.numel(), _s()))
    return y


# ------------------------------------------------------------------ vectors

def _rows(t, name):
    t = _req(t, torch.float32, name)
    B = t.shape[0] if t.dim() > 1 else 1
    return t, B, t.numel() // B


def _vec_work(B, n, dev):
    return torch.empty(int(lib.tspnn_vec_workspace(B, n)) // 4 + 1, dtype=torch.float32,
                       device=dev)


def residual(y, f, diff=None, out=None, active=None):
    """Per object (rows over the leading dimension): res[b] = sum (f - y)^2,
    float32 [B]; diff (like f, may be f itself) receives f - y.  With active
    (bool or int [B] on the device) only the active entries of `out` are
    written, the others keep their values."""
    y, B, n = _rows(y, "y")
    f, B2, n2 = _rows(f, "f")
    if (B, n) != (B2, n2):
        raise ValueError("y and f must have the same shape")
    if diff is not None:
        _req(diff, torch.float32, "diff")
    res = out if out is not None else torch.empty(B, dtype=torch.float32, device=y.device)
    act = None if active is None else active.to(torch.int32).contiguous()
    check(lib.tspnn_residual(_p(y), _p(f), B, n, _p(diff), _p(res), _p(act),
                             _p(_vec_work(B, n, y.device)), _s()))
    return res


def dot(a, b):
    """out[b] = sum a[b] * b[b] per object (float32 [B])."""
    a, B, n = _rows(a, "a")
    b, B2, n2 = _rows(b, "b")
    if (B, n) != (B2, n2):
        raise ValueError("a and b must have the same shape")
    out = torch.empty(B, dtype=torch.float32, device=a.device)
    check(lib.tspnn_dot(_p(a), _p(b), B, n, _p(out), _p(_vec_work(B, n, a.device)), _s()))
    return out


def axpy(x, a, alpha, active=None):
    """x[b] += alpha * a[b] in place, for active objects (all when None)."""
    x, B, n = _rows(x, "x")
    a, B2, n2 = _rows(a, "a")
    if (B, n) != (B2, n2):
        raise ValueError("x and a must have the same shape")
    act = None if active is None else active.to(torch.int32).contiguous()
    check(lib.tspnn_axpy(_p(x), _p(a), float(alpha), B, n, _p(act), _s()))
    return x


def scale(src, alpha, out=None):
    """alpha * src (out may be src itself)."""
    src = _req(src.contiguous(), torch.float32, "src")
    dst = out if out is not None else torch.empty_like(src)
    check(lib.tspnn_scale(_p(src), float(alpha), src.numel(), _p(dst), _s()))
    return dst


# ------------------------------------------------------------------ TV

def tv(rho, eps=1e-6, with_grad=True):
    """Anisotropic smoothed TV of rho (..., D0, D1, D2): returns (value per
    leading index (float32), gradient like rho or None)."""
    rho = _req(rho.contiguous(), torch.float32, "rho")
    D0, D1, D2 = rho.shape[-3:]
    B = int(np.prod(rho.shape[:-3])) if rho.dim() > 3 else 1
    V = D0 * D1 * D2
    work = torch.empty(int(lib.tspnn_tv_workspace(B, V)) // 4 + 1, dtype=torch.float32,
                       device=rho.device)
    val = torch.empty(B, dtype=torch.float32, device=rho.device)
    grad = torch.empty_like(rho) if with_grad else None
    check(lib.tspnn_tv(_p(rho), B, D0, D1, D2, eps, _p(val), _p(grad), _p(work), _s()))
    return val.reshape(rho.shape[:-3]) if rho.dim() > 3 else val[0], grad


class TV(torch.autograd.Function):
    """Differentiable TV(rho) (summed over any leading batch dimensions)."""

    @staticmethod
    def forward(ctx, rho, eps=1e-6):
        val, grad = tv(rho, eps)
        ctx.save_for_backward(grad)
        return val.sum()

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        return scale(grad, float(g)), None


# ------------------------------------------------------------------ Adam

class Adam:
    """Adam (PyTorch semantics, L2 weight decay) over a list of float32 CUDA
    tensors; gradients are passed to step() explicitly."""

    def __init__(self, params, lr=1e-3, betas=(0.9, 0.999), eps=1e-8, weight_decay=0.0):
        self.params = list(params)
        self.lr, self.betas, self.eps, self.wd = lr, betas, eps, weight_decay
        self.m = [torch.zeros_like(p) for p in self.params]
        self.v = [torch.zeros_like(p) for p in self.params]
        self.t = 0

    def state_dict(self):
        """Optimiser state as host arrays (moments per parameter, step count
        and hyper-parameters)."""
        sd = {"t": np.int64(self.t), "lr": np.float64(self.lr),
              "betas": np.asarray(self.betas, np.float64), "eps": np.float64(self.eps),
              "wd": np.float64(self.wd)}
        for k, (m, v) in enumerate(zip(self.m, self.v)):
            sd[f"m{k}"] = m.detach().cpu().numpy()
            sd[f"v{k}"] = v.detach().cpu().numpy()
        return sd

    def load_state_dict(self, sd):
        self.t = int(sd["t"])
        self.lr, self.eps, self.wd = float(sd["lr"]), float(sd["eps"]), float(sd["wd"])
        self.betas = tuple(float(b) for b in np.asarray(sd["betas"]))
        for k, (m, v) in enumerate(zip(self.m, self.v)):
            if tuple(sd[f"m{k}"].shape) != tuple(m.shape):
                raise ValueError(f"moment {k}: shape {sd[f'm{k}'].shape} != {tuple(m.shape)}")
            m.copy_(torch.from_numpy(np.asarray(sd[f"m{k}"])).to(m.device))
            v.copy_(torch.from_numpy(np.asarray(sd[f"v{k}"])).to(v.device))

    def step(self, grads, bf16_copies=None):
        self.t += 1
        for k, (p, g) in enumerate(zip(self.params, grads)):
            _req(p, torch.float32, "param")
            g = _req(g.contiguous(), torch.float32, "grad")
            pb = None if bf16_copies is None else bf16_copies[k]
            check(lib.tspnn_adam(_p(p), _p(g), _p(self.m[k]), _p(self.v[k]), p.numel(), self.lr,
                                 self.betas[0], self.betas[1], self.eps, self.wd, self.t, _p(pb),
                                 _s()))


# ------------------------------------------------------------------ CNN

class CNN:
    """6-layer 3-D CNN on the (r, e, a) grid with a residual output:
        out = x + L5(relu(L4(...relu(L0(x)))))
    L0: 1 -> 32 (FP32 VALU), L1..L4: 32 -> 32 (BF16 MFMA, FP32 accumulate),
    L5: 32 -> 1 (FP32 VALU).  Circular padding in azimuth, zero in r and e.
    Master weights are float32; the 32 -> 32 layers run on bfloat16 copies.
    """

    def __init__(self, channels=32, hidden_layers=4, device="cuda", seed=8, scale_out=0.1):
        assert channels == 32, "the kernels are specialised for 32 channels"
        g = torch.Generator().manual_seed(seed)
        dev = torch.device(device)
        C = channels

        def he(shape, fan_in, s=1.0):
            return (torch.randn(shape, generator=g) * (s * (2.0 / fan_in) ** 0.5)).to(dev)

        self.w0 = he((27, C), 27)
        self.b0 = torch.zeros(C, device=dev)
        self.wh = [he((27, C, C), 27 * C) for _ in range(hidden_layers)]
        self.bh = [torch.zeros(C, device=dev) for _ in range(hidden_layers)]
        self.w5 = he((27, C), 27 * C, scale_out)
        self.b5 = torch.zeros(1, device=dev)
        self.wh_bf = [to_bf16(w) for w in self.wh]
        self.dev = dev
        self._ws = None
        self._acts = None

    # parameters in a fixed order (w0, b0, wh..., bh..., w5, b5)
    def parameters(self):
        return [self.w0, self.b0, *self.wh, *self.bh, self.w5, self.b5]

    def bf16_targets(self):
        n = len(self.wh)
        return [None, None, *self.wh_bf, *([None] * n), None, None]

    def state_dict(self):
        return {f"p{i}": p.detach().cpu().numpy() for i, p in enumerate(self.parameters())}

    def load_state_dict(self, sd):
        for i, p in enumerate(self.parameters()):
            p.copy_(torch.from_numpy(np.asarray(sd[f"p{i}"])).to(p.device))
        self.wh_bf = [to_bf16(w) for w in self.wh]

    def _workspace(self, N, D):
        need = int(lib.tspnn_conv_workspace(N, *D)) // 4 + 1
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.float32, device=self.dev)
        return self._ws

    def forward(self, x, keep=True):
        """x: (N, D0, D1, D2) float32 on the GPU -> (N, D0, D1, D2) float32."""
        x = _req(x.contiguous(), torch.float32, "x")
        N, D0, D1, D2 = x.shape
        C = 32
        acts = [torch.empty((N, D0, D1, D2, C), dtype=torch.bfloat16, device=self.dev)]
        check(lib.tspnn_conv_in_fwd(_p(x), N, D0, D1, D2, _p(self.w0), _p(self.b0),
                                    _p(acts[0]), _s()))
        for w, b in zip(self.wh_bf, self.bh):
            a = torch.empty_like(acts[-1])
            check(lib.tspnn_conv_fwd(_p(acts[-1]), N, D0, D1, D2, _p(w), _p(b), _p(a), _s()))
            acts.append(a)
        out = torch.empty_like(x)
        check(lib.tspnn_conv_out_fwd(_p(acts[-1]), N, D0, D1, D2, _p(self.w5), _p(self.b5), _p(x),
                                     _p(out), _s()))
        self._acts = (x, acts) if keep else None
        return out

    __call__ = forward

    def backward(self, dout, keep=False):
        """Gradients of sum(dout * out) with respect to the parameters, in
        parameters() order, after forward(..., keep=True).  keep=True also
        keeps the gradients reaching each layer's pre-activation (the dz of
        layers 0 .. 4, bfloat16) in self.dz, for inspection."""
        x, acts = self._acts
        dout = _req(dout.contiguous(), torch.float32, "dout")
        N, D0, D1, D2 = x.shape
        ws = self._workspace(N, (D0, D1, D2))
        n = len(self.wh)
        gw = [None] * n
        gb = [None] * n
        dw5 = torch.empty_like(self.w5)
        db5 = torch.empty_like(self.b5)
        dz = torch.empty_like(acts[-1])
        check(lib.tspnn_conv_out_bwd(_p(acts[-1]), _p(dout), N, D0, D1, D2, _p(self.w5), _p(dw5),
                                     _p(db5), _p(dz), _p(ws), _s()))
        kept = [dz]
        for k in range(n - 1, -1, -1):
            # layer k maps acts[k] -> acts[k+1]; dz = dL/d(pre-activation of layer k)
            gw[k] = torch.empty_like(self.wh[k])
            gb[k] = torch.empty_like(self.bh[k])
            check(lib.tspnn_conv_bwd_weight(_p(acts[k]), _p(dz), N, D0, D1, D2, _p(gw[k]),
                                            _p(gb[k]), _p(ws), _s()))
            wt = torch.empty_like(self.wh_bf[k])
            check(lib.tspnn_conv_flip_weights(_p(self.wh_bf[k]), _p(wt), _s()))
            dz_prev = torch.empty_like(dz)
            check(lib.tspnn_conv_bwd_data(_p(dz), N, D0, D1, D2, _p(wt), _p(acts[k]),
                                          _p(dz_prev), _s()))
            dz = dz_prev
            kept.append(dz)
        self.dz = kept[::-1] if keep else None
        dw0 = torch.empty_like(self.w0)
        db0 = torch.empty_like(self.b0)
        check(lib.tspnn_conv_in_bwd_weight(_p(x), _p(dz), N, D0, D1, D2, _p(dw0), _p(db0),
                                           _p(ws), _s()))
        return [dw0, db0, *gw, *gb, dw5, db5]


# ------------------------------------------------------------------ measurement

def stream_copy(src, dst, blocks=4096):
    """dst <- src by the library's streaming copy kernel (float32, 16-byte aligned)."""
    check(lib.tspnn_stream_copy(_p(_req(src, torch.float32, "src")),
                                _p(_req(dst, torch.float32, "dst")), src.numel(), blocks, _s()))


def stream_read(src, partial, blocks=4096):
    """Read every element of src; per-block sums into partial[:blocks]."""
    check(lib.tspnn_stream_read(_p(_req(src, torch.float32, "src")), src.numel(), blocks,
                                _p(_req(partial, torch.float32, "partial")), _s()))


# ------------------------------------------------------------------ checkpoints

def save_checkpoint(path, net, opt=None, **extra):
    """Write the CNN's FP32 master weights, the optimiser state (if given)
    and extra scalars to an .npz file (plain arrays, no pickled objects)."""
    arrs = {f"net_{k}": v for k, v in net.state_dict().items()}
    if opt is not None:
        arrs.update({f"opt_{k}": v for k, v in opt.state_dict().items()})
    arrs.update({f"extra_{k}": np.asarray(v) for k, v in extra.items()})
    np.savez(path, **arrs)


def load_checkpoint(path, net, opt=None):
    """Restore what save_checkpoint wrote (the BF16 weight copies are
    re-derived from the masters); returns the extra scalars."""
    with np.load(path, allow_pickle=False) as z:
        net.load_state_dict({k[4:]: z[k] for k in z.files if k.startswith("net_")})
        if opt is not None:
            opt.load_state_dict({k[4:]: z[k] for k in z.files if k.startswith("opt_")})
        return {k[6:]: z[k][()] for k in z.files if k.startswith("extra_")}

