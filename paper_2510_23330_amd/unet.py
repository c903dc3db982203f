"""3-D U-Net surrogate (Sec. 3.3) composed from libgx's BF16-MFMA blocks.

Architecture (the paper's figure is not available; these choices are stated
in the design notes): 4 levels with 32, 64, 128, 256 channels; two 3^3
convolutions (zero padding 1, bias, LeakyReLU 0.1) per level on the way down
and up; 2^3 average pooling down; nearest x2 upsampling followed by a 3^3
convolution on the way up; skip connections by channel concatenation; a
linear 1^3 head.  Inputs carry 5 physical channels padded to 8, outputs 5
channels padded to 16 (FP32).  Activations and weights are BF16, every
convolution accumulates in FP32; master weights and Adam moments are FP32.

This module sequences libgx calls and owns the parameter/activation buffers;
all arithmetic runs in libgx kernels.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

CIN_PAD = 8
COUT_PAD = 16
N_CHAN = 5


@dataclass
class Layer:
    name: str
    cin: int
    cout: int
    ksize: int
    act: bool
    w_off: int = 0
    b_off: int = 0

    @property
    def kvol(self):
        return 27 if self.ksize == 3 else 1

    @property
    def n_w(self):
        return self.cout * self.kvol * self.cin


def layers(base: int = 32, levels: int = 4):
    ch = [base * 2 ** l for l in range(levels)]
    L = []
    cin = CIN_PAD
    for l in range(levels):
        L.append(Layer(f"e{l}a", cin, ch[l], 3, True))
        L.append(Layer(f"e{l}b", ch[l], ch[l], 3, True))
        cin = ch[l]
    for l in range(levels - 2, -1, -1):
        L.append(Layer(f"u{l}c", ch[l + 1], ch[l], 3, True))
        L.append(Layer(f"d{l}a", 2 * ch[l], ch[l], 3, True))
        L.append(Layer(f"d{l}b", ch[l], ch[l], 3, True))
    L.append(Layer("head", ch[0], COUT_PAD, 1, False))
    off = 0
    for ly in L:
        ly.w_off = off
        off += ly.n_w
    for ly in L:
        ly.b_off = off
        off += ly.cout
    return L, off


def flops_forward(S: int, base: int = 32, levels: int = 4) -> float:
    """Multiply-add count x 2 of one forward pass of one sample (padded channels)."""
    L, _ = layers(base, levels)
    tot = 0.0
    for ly in L:
        if ly.name.startswith("e"):
            lev = int(ly.name[1])
        elif ly.name == "head":
            lev = 0
        else:
            lev = int(ly.name[1])
        vox = (S // 2 ** lev) ** 3
        tot += 2.0 * vox * ly.kvol * ly.cin * ly.cout
    return tot


class UNet:
    def __init__(self, eng, S: int = 64, batch: int = 4, base: int = 32, levels: int = 4,
                 seed: int = 0, device="cuda", train: bool = True):
        import torch
        self.torch = torch
        self.eng = eng
        self.S, self.B, self.levels = S, batch, levels
        self.ch = [base * 2 ** l for l in range(levels)]
        self.L, n = layers(base, levels)
        self.by = {ly.name: ly for ly in self.L}
        self.n_params = n
        rng = np.random.Generator(np.random.PCG64(seed))
        w = np.zeros(n, np.float32)
        for ly in self.L:
            fan_in = ly.kvol * ly.cin
            bound = math.sqrt(6.0 / fan_in) if ly.act else math.sqrt(3.0 / fan_in)
            w[ly.w_off:ly.w_off + ly.n_w] = rng.uniform(-bound, bound, ly.n_w)
        if True:  # padded input channels and padded head outputs carry nothing
            for ly in self.L:
                if ly.name == "e0a":
                    ww = w[ly.w_off:ly.w_off + ly.n_w].reshape(ly.cout, ly.kvol, ly.cin)
                    ww[:, :, N_CHAN:] = 0
                if ly.name == "head":
                    ww = w[ly.w_off:ly.w_off + ly.n_w].reshape(ly.cout, ly.kvol, ly.cin)
                    ww[N_CHAN:] = 0
        f32 = dict(dtype=torch.float32, device=device)
        self.w32 = torch.as_tensor(w, **f32)
        self.grad = torch.zeros(n, **f32)
        self.m = torch.zeros(n, **f32)
        self.v = torch.zeros(n, **f32)
        self.wbf = torch.zeros(n, dtype=torch.bfloat16, device=device)
        eng.f32_to_bf16(self.w32, self.wbf)
        self.t = 0
        self.device = device
        self.train_mode = train
        self.acts = {}
        self._alloc(batch)

    # ---- buffers --------------------------------------------------------------
    def _alloc(self, B):
        torch = self.torch
        S, ch = self.S, self.ch
        bf = dict(dtype=torch.bfloat16, device=self.device)
        A = {}
        for l in range(self.levels):
            s = S // 2 ** l
            A[f"e{l}a"] = torch.zeros(B * s ** 3 * ch[l], **bf)
            A[f"e{l}b"] = torch.zeros(B * s ** 3 * ch[l], **bf)
            if l < self.levels - 1:
                A[f"p{l}"] = torch.zeros(B * (s // 2) ** 3 * ch[l], **bf)
        for l in range(self.levels - 2, -1, -1):
            s = S // 2 ** l
            if self.train_mode:  # inference reads them through the fused convolution
                A[f"up{l}"] = torch.zeros(B * s ** 3 * ch[l + 1], **bf)
                A[f"c{l}"] = torch.zeros(B * s ** 3 * 2 * ch[l], **bf)
            A[f"u{l}c"] = torch.zeros(B * s ** 3 * ch[l], **bf)
            A[f"d{l}a"] = torch.zeros(B * s ** 3 * ch[l], **bf)
            A[f"d{l}b"] = torch.zeros(B * s ** 3 * ch[l], **bf)
        self.pred = torch.zeros(B * S ** 3 * COUT_PAD, dtype=torch.float32, device=self.device)
        self.acts = A
        if self.train_mode:
            self.G = {k: torch.zeros_like(v) for k, v in A.items()}
            self.G["skip"] = {l: torch.zeros(B * (S // 2 ** l) ** 3 * ch[l], **bf)
                              for l in range(self.levels - 1)}
            self.dpred = torch.zeros(B * S ** 3 * COUT_PAD, **bf)
        else:
            self.G, self.dpred = None, None
        self.Bcur = B

    def _w(self, ly):
        return self.wbf[ly.w_off:ly.w_off + ly.n_w]

    def _b(self, ly):
        return self.w32[ly.b_off:ly.b_off + ly.cout]

    def _conv(self, name, x, S, out_bf=None, out_f32=None):
        ly = self.by[name]
        self.eng.conv3d_fwd(x, self.Bcur, S, ly.cin, self._w(ly), self._b(ly), ly.ksize, ly.cout,
                            ly.act, out_bf16=out_bf, out_f32=out_f32)

    def _conv_fused(self, name, x, c1, x2, up, S, out_bf):
        ly = self.by[name]
        self.eng.conv3d_fwd_fused(x, c1, x2, up, self.Bcur, S, ly.cin, self._w(ly), self._b(ly),
                                  ly.cout, ly.act, out_bf16=out_bf)

    # ---- forward ----------------------------------------------------------------
    def forward(self, x, out_phys=None, scale=None, shift=None):
        """x: bf16 [B * S^3 * 8] standardized input; returns fp32 [B * S^3 * 16].
        With out_phys (fp32 [B * S^3 * 5]) the head writes the first five
        outputs mapped by scale * y + shift there instead, and returns it."""
        A, S, ch, B = self.acts, self.S, self.ch, self.Bcur
        h = x
        for l in range(self.levels):
            s = S // 2 ** l
            self._conv(f"e{l}a", h, s, A[f"e{l}a"])
            if l < self.levels - 1:  # the pooled copy comes from the same launch
                ly = self.by[f"e{l}b"]
                self.eng.conv3d_fwd_pool(A[f"e{l}a"], B, s, ly.cin, self._w(ly), self._b(ly),
                                         ly.cout, ly.act, A[f"e{l}b"], A[f"p{l}"])
                h = A[f"p{l}"]
            else:
                self._conv(f"e{l}b", A[f"e{l}a"], s, A[f"e{l}b"])
        h = A[f"e{self.levels - 1}b"]
        for l in range(self.levels - 2, -1, -1):
            s = S // 2 ** l
            if self.train_mode:
                # the backward pass needs the upsampled and concatenated inputs
                self.eng.upsample2(h, B, s // 2, ch[l + 1], A[f"up{l}"])
                self._conv(f"u{l}c", A[f"up{l}"], s, A[f"u{l}c"])
                self.eng.concat(A[f"u{l}c"], ch[l], A[f"e{l}b"], ch[l], B * s ** 3, A[f"c{l}"])
                self._conv(f"d{l}a", A[f"c{l}"], s, A[f"d{l}a"])
            else:
                self._conv_fused(f"u{l}c", h, ch[l + 1], None, 1, s, A[f"u{l}c"])
                self._conv_fused(f"d{l}a", A[f"u{l}c"], ch[l], A[f"e{l}b"], 0, s, A[f"d{l}a"])
            self._conv(f"d{l}b", A[f"d{l}a"], s, A[f"d{l}b"])
            h = A[f"d{l}b"]
        if out_phys is not None:
            ly = self.by["head"]
            self.eng.conv_head(h, B, S, ly.cin, self._w(ly), self._b(ly), ly.cout, N_CHAN, scale,
                               shift, out_phys, N_CHAN)
            return out_phys
        self._conv("head", h, S, out_f32=self.pred)
        return self.pred

    # ---- backward ---------------------------------------------------------------
    def _wgrad(self, name, x, dy, S):
        ly = self.by[name]
        self.eng.conv3d_bwd_weight(x, dy, self.Bcur, S, ly.cin, ly.ksize, ly.cout,
                                   self.grad[ly.w_off:ly.w_off + ly.n_w],
                                   self.grad[ly.b_off:ly.b_off + ly.cout])

    def _dgrad(self, name, dy, S, y_in, dx):
        ly = self.by[name]
        self.eng.conv3d_bwd_data(dy, self.Bcur, S, ly.cin, self._w(ly), ly.ksize, ly.cout, y_in, dx)

    def backward(self, x, dpred):
        """Accumulate parameter gradients for input x and dL/dpred (bf16)."""
        A, Gd, S, ch, B = self.acts, self.G, self.S, self.ch, self.Bcur
        eng = self.eng
        top = self.levels - 1
        # head
        self._wgrad("head", A["d0b"], dpred, S)
        self._dgrad("head", dpred, S, A["d0b"], Gd["d0b"])
        # decoder, finest level first
        for l in range(0, top):
            s = S // 2 ** l
            self._wgrad(f"d{l}b", A[f"d{l}a"], Gd[f"d{l}b"], s)
            self._dgrad(f"d{l}b", Gd[f"d{l}b"], s, A[f"d{l}a"], Gd[f"d{l}a"])
            self._wgrad(f"d{l}a", A[f"c{l}"], Gd[f"d{l}a"], s)
            self._dgrad(f"d{l}a", Gd[f"d{l}a"], s, None, Gd[f"c{l}"])
            eng.concat(Gd[f"u{l}c"], ch[l], Gd["skip"][l], ch[l], B * s ** 3, Gd[f"c{l}"], split=True)
            eng.grad_combine(Gd[f"u{l}c"], None, A[f"u{l}c"], Gd[f"u{l}c"])
            self._wgrad(f"u{l}c", A[f"up{l}"], Gd[f"u{l}c"], s)
            self._dgrad(f"u{l}c", Gd[f"u{l}c"], s, None, Gd[f"up{l}"])
            # into the next coarser level's output
            below = f"d{l + 1}b" if l + 1 < top else f"e{top}b"
            eng.upsample2(Gd[f"up{l}"], B, s // 2, ch[l + 1], Gd[below], backward=True)
            eng.grad_combine(Gd[below], None, A[below], Gd[below])
        # encoder, coarsest level first
        for l in range(top, -1, -1):
            s = S // 2 ** l
            self._wgrad(f"e{l}b", A[f"e{l}a"], Gd[f"e{l}b"], s)
            self._dgrad(f"e{l}b", Gd[f"e{l}b"], s, A[f"e{l}a"], Gd[f"e{l}a"])
            if l == 0:
                self._wgrad("e0a", x, Gd["e0a"], s)
                break
            self._wgrad(f"e{l}a", A[f"p{l - 1}"], Gd[f"e{l}a"], s)
            self._dgrad(f"e{l}a", Gd[f"e{l}a"], s, None, Gd[f"p{l - 1}"])
            # through the pooling into level l-1's output, plus its skip gradient
            eng.avgpool2(Gd[f"p{l - 1}"], B, 2 * s, ch[l - 1], Gd[f"e{l - 1}b"], backward=True)
            eng.grad_combine(Gd[f"e{l - 1}b"], Gd["skip"][l - 1], A[f"e{l - 1}b"],
                             Gd[f"e{l - 1}b"])

    def zero_grad(self):
        self.grad.zero_()

    def adam(self, lr=1e-4, b1=0.9, b2=0.999, eps=1e-8):
        self.t += 1
        self.eng.adam_step(self.w32, self.grad, self.m, self.v, lr, b1, b2, eps, self.t, self.wbf)

    def train_step(self, x, target, lr=1e-4):
        """One minibatch: forward, MSE, backward, Adam.  Returns the loss."""
        self.forward(x)
        V = self.Bcur * self.S ** 3
        loss = self.eng.mse(self.pred, COUT_PAD, target, N_CHAN, V, self.dpred)
        self.zero_grad()
        self.backward(x, self.dpred)
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
