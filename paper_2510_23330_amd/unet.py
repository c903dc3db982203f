"""3-D U-Net surrogate (Sec. 3.3) on libgx's whole-network calls.

Architecture (the paper's figure is not available; these choices are stated
in the design notes): 4 levels with 32, 64, 128, 256 channels; two 3^3
convolutions (zero padding 1, bias, LeakyReLU 0.1) per level on the way down
and up; 2^3 average pooling down; nearest x2 upsampling followed by a 3^3
convolution on the way up; skip connections by channel concatenation; a
linear 1^3 head.  Inputs carry nc_in channels padded to 8 (5 physical
channels, or the 8 cubes of the paper's encoding), outputs nc_out channels
padded to 16 (FP32).  Activations and weights are BF16, every
convolution accumulates in FP32; master weights and Adam moments are FP32.

The layer sequence of each pass runs inside the library (gx_unet_forward,
gx_unet_backward, which also hold the activations); this module owns the
parameter, gradient, moment and output buffers and marshals the calls.  The
layer table (names, channels, offsets) comes from the library too.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

CIN_PAD = 8
COUT_PAD = 16


@dataclass
class Layer:
    name: str
    cin: int
    cout: int
    ksize: int
    w_off: int
    b_off: int

    @property
    def act(self):
        return self.name != "head"

    @property
    def kvol(self):
        return 27 if self.ksize == 3 else 1

    @property
    def n_w(self):
        return self.cout * self.kvol * self.cin


def layers(base: int = 32, levels: int = 4):
    """The library's layer table and the total parameter count."""
    from . import unet_layers, unet_sizes
    L = [Layer(*t) for t in unet_layers(levels, base, CIN_PAD, COUT_PAD)]
    n, _ = unet_sizes(levels, base, CIN_PAD, COUT_PAD)
    return L, n


def flops_forward(S: int, base: int = 32, levels: int = 4) -> float:
    """Multiply-add count x 2 of one forward pass of one sample (padded channels)."""
    L, _ = layers(base, levels)
    tot = 0.0
    for ly in L:
        lev = 0 if ly.name == "head" else int(ly.name[1])
        vox = (S // 2 ** lev) ** 3
        tot += 2.0 * vox * ly.kvol * ly.cin * ly.cout
    return tot


ACT_NAMES = ("e{l}a", "e{l}b", "p{l}", "up{l}", "u{l}c", "c{l}", "d{l}a", "d{l}b")


class UNet:
    def __init__(self, eng, S: int = 64, batch: int = 4, base: int = 32, levels: int = 4,
                 seed: int = 0, device="cuda", train: bool = True, nc_in: int = 5,
                 nc_out: int = 5):
        if not (1 <= nc_in <= CIN_PAD and 1 <= nc_out <= COUT_PAD):
            raise ValueError("channel counts exceed the padded widths")
        import torch
        self.torch = torch
        self.eng = eng
        self.S, self.B, self.levels, self.base = S, batch, levels, base
        self.nc_in, self.nc_out = nc_in, nc_out
        self.ch = [base * 2 ** l for l in range(levels)]
        self.L, n = layers(base, levels)
        self.by = {ly.name: ly for ly in self.L}
        self.n_params = n
        rng = np.random.Generator(np.random.PCG64(seed))
        w = np.zeros(n, np.float32)
        for ly in self.L:
            fan_in = ly.kvol * ly.cin
            bound = math.sqrt(6.0 / fan_in) if ly.act else math.sqrt(3.0 / fan_in)
            ww = rng.uniform(-bound, bound, ly.n_w).reshape(ly.cout, ly.kvol, ly.cin)
            # padded input channels and padded head outputs carry nothing
            if ly.name == "e0a":
                ww[:, :, nc_in:] = 0
            if ly.name == "head":
                ww[nc_out:] = 0
            w[ly.w_off:ly.w_off + ly.n_w] = ww.ravel()
        f32 = dict(dtype=torch.float32, device=device)
        self.w32 = torch.as_tensor(w, **f32)
        self.grad = torch.zeros(n, **f32)
        self.m = torch.zeros(n, **f32)
        self.v = torch.zeros(n, **f32)
        self.wbf = torch.zeros(n, dtype=torch.bfloat16, device=device)
        eng.f32_to_bf16(self.w32, self.wbf)
        self.desc = eng._unet_desc(levels, base, CIN_PAD, COUT_PAD, self.wbf, self.w32)
        self.t = 0
        self.device = device
        self.train_mode = train
        self.pred = torch.zeros(batch * S ** 3 * COUT_PAD, **f32)
        self.dpred = torch.zeros(batch * S ** 3 * COUT_PAD, dtype=torch.bfloat16,
                                 device=device) if train else None
        self.Bcur = batch

    # ---- forward ----------------------------------------------------------------
    def forward(self, x, out_phys=None, scale=None, shift=None):
        """x: bf16 [Bcur * S^3 * 8] standardized input; returns fp32 [Bcur * S^3 * 16].
        With out_phys (fp32 [Bcur * S^3 * nc_out]) the head writes the first
        nc_out outputs mapped by scale * y + shift there instead, and returns it.  A
        training-mode network keeps its activations for backward()."""
        B, S = self.Bcur, self.S
        if out_phys is not None:
            self.eng.unet_forward(self.desc, x, B, S, self.train_mode, None, self.nc_out, scale,
                                  shift, out_phys)
            return out_phys
        out = self.pred[:B * S ** 3 * COUT_PAD]
        self.eng.unet_forward(self.desc, x, B, S, self.train_mode, out_f32=out)
        return out

    @property
    def acts(self):
        """The activations kept by the last training-mode forward pass."""
        out = {}
        for l in range(self.levels):
            for pat in ACT_NAMES:
                name = pat.format(l=l)
                if (pat in ("e{l}a", "e{l}b") or l < self.levels - 1):
                    out[name] = self.eng.unet_saved(name)
        return out

    # ---- backward ---------------------------------------------------------------
    def backward(self, x, dpred):
        """Accumulate parameter gradients for input x and dL/dpred (bf16)."""
        self.eng.unet_backward(self.desc, x, self.Bcur, self.S, dpred, self.grad)

    def zero_grad(self):
        self.grad.zero_()

    def adam(self, lr=1e-4, b1=0.9, b2=0.999, eps=1e-8):
        self.t += 1
        self.eng.adam_step(self.w32, self.grad, self.m, self.v, lr, b1, b2, eps, self.t, self.wbf)

    def train_step(self, x, target, lr=1e-4):
        """One minibatch: forward, MSE, backward, Adam.  Returns the loss."""
        pred = self.forward(x)
        V = self.Bcur * self.S ** 3
        dp = self.dpred[:V * COUT_PAD]
        loss = self.eng.mse(pred, COUT_PAD, target, self.nc_out, V, dp)
        self.zero_grad()
        self.backward(x, dp)
        self.adam(lr)
        return loss

    def state_dict(self):
        return {"w32": self.w32.cpu().numpy(), "m": self.m.cpu().numpy(),
                "v": self.v.cpu().numpy(), "t": self.t}

    def load_state_dict(self, d):
        torch = self.torch
        self.w32.copy_(torch.as_tensor(d["w32"]))
        self.m.copy_(torch.as_tensor(d["m"]))
        self.v.copy_(torch.as_tensor(d["v"]))
        self.t = int(d["t"])
        self.eng.f32_to_bf16(self.w32, self.wbf)
