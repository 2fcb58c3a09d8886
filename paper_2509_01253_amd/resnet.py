"""ResNet-18-shaped stack of encrypted linear layers (one server round per layer).

Paper Sec. 4: each round the server evaluates one linear layer on the client's
fresh ciphertexts, the client decrypts, applies the non-linearity in the clear
and re-encrypts.  For a ResNet-18 on H x W x 3 inputs (3x3 stride-1 stem, no
max-pool) the server sees 21 layers: the stem, 16 block convolutions, three
1x1 downsampling convolutions and the final FC.  Strided convolutions are
evaluated at stride 1 on the input resolution and the client keeps every second
row and column when it reads the output; batch norm is folded into the conv
weights; residual additions, ReLU and the global average pool run on the
client between rounds.

This module holds the layer list, the FP64 plaintext forward pass (the client
side and the reference), and `EncryptedStack`, which runs the server side on
the GPU through the fhelin ABI with one captured graph per layer schedule.
Encryption and decryption are supplied by the caller (the client).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class LayerSpec:
    name: str
    kind: str           # "conv" or "fc"
    c_in: int
    c_out: int
    h: int              # input (= evaluated) resolution
    w: int
    k: int = 3          # conv kernel
    stride: int = 1     # client-side subsampling of the output
    fc_n: int = 0       # padded FC size


def resnet18_layers(h: int = 64, w: int = 64, c0: int = 3, widths=(64, 128, 256, 512), n_classes: int = 200):
    L = [LayerSpec("stem", "conv", c0, widths[0], h, w)]
    c, hh, ww = widths[0], h, w
    for s, cw in enumerate(widths):
        for blk in range(2):
            stride = 2 if (s > 0 and blk == 0) else 1
            L.append(LayerSpec(f"s{s + 1}b{blk + 1}c1", "conv", c, cw, hh, ww, 3, stride))
            oh, ow = hh // stride, ww // stride
            L.append(LayerSpec(f"s{s + 1}b{blk + 1}c2", "conv", cw, cw, oh, ow, 3, 1))
            if stride == 2:
                L.append(LayerSpec(f"s{s + 1}b{blk + 1}ds", "conv", c, cw, hh, ww, 1, 2))
            c, hh, ww = cw, oh, ow
    n = 1
    while n < max(c, n_classes):
        n *= 2
    L.append(LayerSpec("fc", "fc", c, n_classes, 1, 1, fc_n=n))
    return L


def conv_channel_babies(spec: LayerSpec, slots: int) -> int:
    """Channel baby steps for a conv layer's plan.  Each channel offset that becomes a
    baby step trades a giant-step key switch (ModDown, ModUp, their transforms) for a
    hoisted rotation (an inner product), but the multiply-accumulate then reads
    n1 times as many rotated inputs for every output ciphertext.  Measured on the
    ResNet-18 stack at N = 2^16: with 8 or 32 channels per ciphertext the split was
    slower or even (up to 3.5x slower for 8 in / 8 out ciphertexts), with 128 or 512
    it was 2-3x faster.  So: no split below 64 channels per ciphertext, else the
    largest power of two n1 dividing them with n1 k^2 <= 64 (the plan's limit)."""
    cct = slots // (spec.h * spec.w)
    n1 = 1
    if cct < 64:
        return n1
    while cct % (2 * n1) == 0 and 2 * n1 * spec.k * spec.k <= 64:
        n1 *= 2
    return n1


def shuffle_perms(specs, stream) -> dict:
    """Seeded channel (conv) / neuron (FC) permutations of every layer, as
    {name: (perm_out, perm_in)} for fhelin_plan_encode_weights (paper Sec. 4.4:
    each round's weights fold this round's shuffle sigma_r of the outputs and the
    unshuffle sigma_{r-1}^-1 of the previous round's outputs).

    The client holds every activation in its shuffled order a'[t] = a[sigma[t]]
    and never learns sigma: ReLU, the stride subsampling and the average pool act
    per channel and commute with a channel permutation.  A residual addition needs
    both operands under the same permutation, so the conv whose output is added to
    a block's skip path (c2) takes the skip path's permutation: the block input's
    in an identity block, the downsampling conv's (drawn fresh) otherwise.  The
    stem's input is the image in its own order (sigma_0 = id) and the final FC's
    output is not shuffled (the client reads the logits; paper Sec. 5)."""
    perm = {}
    cur = None  # permutation of the activation entering the next layer (None = identity)
    by = {s.name: s for s in specs}
    order = [s.name for s in specs]
    stem = by["stem"]
    perm["stem"] = (stream.permutation(stem.c_out), None)
    cur = perm["stem"][0]
    names = order[1:-1]
    i = 0
    while i < len(names):
        c1, c2 = by[names[i]], by[names[i + 1]]
        ds = by[names[i + 2]] if i + 2 < len(names) and names[i + 2].endswith("ds") else None
        p1 = stream.permutation(c1.c_out)
        perm[c1.name] = (p1, cur)
        if ds is not None:
            pskip = stream.permutation(ds.c_out)
            perm[ds.name] = (pskip, cur)
            i += 3
        else:
            pskip = cur
            i += 2
        perm[c2.name] = (pskip, p1)
        cur = pskip
    perm["fc"] = (None, cur)
    return perm


def init_weights(specs, stream) -> dict:
    """He-normal weights (batch norm folded), seeded."""
    W = {}
    for sp in specs:
        if sp.kind == "conv":
            W[sp.name] = stream.he_normal((sp.c_out, sp.c_in, sp.k, sp.k), sp.c_in * sp.k * sp.k)
        else:
            W[sp.name] = stream.he_normal((sp.c_out, sp.c_in), sp.c_in)
    return W


def conv_same(W: np.ndarray, x: np.ndarray) -> np.ndarray:
    """FP64 'same' convolution, stride 1 (cross-correlation, zero padding k//2)."""
    c_out, c_in, k, _ = W.shape
    r = k // 2
    _, h, w = x.shape
    xp = np.zeros((c_in, h + 2 * r, w + 2 * r))
    xp[:, r:r + h, r:r + w] = x
    y = np.zeros((c_out, h, w))
    for dy in range(k):
        for dx in range(k):
            y += np.tensordot(W[:, :, dy, dx], xp[:, dy:dy + h, dx:dx + w], axes=(1, 0))
    return y


class Forward:
    """The network as a sequence of server rounds.  `linear(spec, x)` is the
    server's layer (plaintext here, encrypted in EncryptedStack); everything
    else is the client's work between rounds."""

    def __init__(self, specs, weights):
        self.specs = {s.name: s for s in specs}
        self.order = [s.name for s in specs]
        self.W = weights

    def run(self, x: np.ndarray, linear) -> np.ndarray:
        sp = self.specs
        h = np.maximum(linear(sp["stem"], x), 0.0)
        names = self.order[1:-1]
        i = 0
        while i < len(names):
            c1, c2 = names[i], names[i + 1]
            ds = names[i + 2] if i + 2 < len(names) and names[i + 2].endswith("ds") else None
            s1 = sp[c1]
            a = linear(s1, h)
            if s1.stride == 2:
                a = a[:, ::2, ::2]
            a = np.maximum(a, 0.0)
            b = linear(sp[c2], a)
            if ds:
                sc = linear(sp[ds], h)[:, ::2, ::2]
                i += 3
            else:
                sc = h
                i += 2
            h = np.maximum(b + sc, 0.0)
        pooled = h.mean(axis=(1, 2))
        return linear(sp["fc"], pooled)

    def plain_linear(self, spec: LayerSpec, x: np.ndarray) -> np.ndarray:
        if spec.kind == "conv":
            return conv_same(self.W[spec.name], x)
        return self.W[spec.name] @ x


class EncryptedStack:
    """Server side of the stack on the GPU: per layer a plan, GPU-encoded weights,
    the client's Galois keys, and a captured graph of the layer schedule (one per
    layer; replayed every inference).

    client.encrypt(slots [n][S], level) -> [n][2][level][N] device tensor,
    client.decrypt(ct tensor, level, scale) -> [n][S] real slots, and
    client.keys(galois list, level) -> evk device tensor in the ABI layout."""

    def __init__(self, F, ctx, log_n, specs, weights, client, level: int, scale: float, q_level_top: int,
                 flags, stream, perms=None):
        import torch

        self.F, self.ctx, self.torch = F, ctx, torch
        self.S = 1 << (log_n - 1)
        self.N = 1 << log_n
        self.level, self.scale, self.flags, self.stream = level, scale, flags, stream
        self.out_scale = scale * scale / q_level_top
        self.client = client
        self.layers = {}
        for sp in specs:
            if sp.kind == "conv":
                plan = F.fhelin_plan_create(ctx, F.FHELIN_LAYER_CONV, c_in=sp.c_in, c_out=sp.c_out, h=sp.h, w=sp.w,
                                            k=sp.k)
            else:
                plan = F.fhelin_plan_create(ctx, F.FHELIN_LAYER_FC, fc_n=sp.fc_n, fc_out=sp.c_out, fc_in=sp.c_in,
                                            n1=min(16, sp.fc_n))
            info = F.fhelin_plan_info(plan)
            Wd = torch.from_numpy(np.ascontiguousarray(weights[sp.name])).cuda()
            po, pi = (perms or {}).get(sp.name, (None, None))
            po = None if po is None else torch.from_numpy(np.ascontiguousarray(po, np.int32)).cuda()
            pi = None if pi is None else torch.from_numpy(np.ascontiguousarray(pi, np.int32)).cuda()
            pts = F.fhelin_plan_encode_weights(ctx, plan, Wd, po, pi, level, scale)
            gal = F.fhelin_plan_galois(plan)
            ks = F.fhelin_keyset_load(ctx, gal, level, client.keys(gal, level)) if gal else None
            x = torch.zeros((info["n_in"], 2, level, self.N), dtype=torch.int64, device="cuda")
            y = torch.zeros((info["n_out"], 2, level, self.N), dtype=torch.int64, device="cuda")
            self.layers[sp.name] = dict(spec=sp, plan=plan, info=info, pts=pts, ks=ks, x=x, y=y, graph=None)

    def _graph(self, L):
        if L["graph"] is None:
            F, torch = self.F, self.torch
            lv = [self.level] * L["info"]["n_in"]
            ol = [self.level - 1] * L["info"]["n_out"]
            torch.cuda.synchronize()
            with torch.cuda.stream(self.stream):
                L["graph"] = F.fhelin_graph_capture_linear(self.ctx, L["plan"], L["ks"], L["pts"], L["x"], lv, L["y"],
                                                           ol, self.flags, stream=self.stream)
        return L["graph"]

    def pack(self, spec: LayerSpec, x: np.ndarray) -> np.ndarray:
        """Client-side slot packing of a layer input."""
        S = self.S
        if spec.kind == "fc":
            xn = np.zeros(spec.fc_n)
            xn[: x.size] = x
            return np.tile(xn, S // spec.fc_n)[None]
        cct = S // (spec.h * spec.w)
        n_in = -(-spec.c_in // cct)
        buf = np.zeros((n_in * cct, spec.h, spec.w))
        buf[: spec.c_in] = x
        return buf.reshape(n_in, S)

    def unpack(self, spec: LayerSpec, z: np.ndarray) -> np.ndarray:
        if spec.kind == "fc":
            return z[0][: spec.c_out]
        return z.reshape(-1, spec.h, spec.w)[: spec.c_out]

    def linear(self, spec: LayerSpec, x: np.ndarray) -> np.ndarray:
        """One round: client encrypts, server replays the layer graph, client decrypts."""
        L = self.layers[spec.name]
        ct = self.client.encrypt(self.pack(spec, x), self.level)
        L["x"].copy_(ct)
        self.torch.cuda.synchronize()
        self.F.fhelin_graph_launch(self._graph(L), stream=self.stream)
        self.stream.synchronize()
        z = self.client.decrypt(L["y"], self.level - 1, self.out_scale)
        return self.unpack(spec, z)

    def close(self):
        F = self.F
        self.torch.cuda.synchronize()
        for L in self.layers.values():
            if L["graph"] is not None:
                F.fhelin_graph_destroy(L["graph"])
            F.fhelin_ptset_release(L["pts"])
            if L["ks"] is not None:
                F.fhelin_keyset_release(L["ks"])
            F.fhelin_plan_destroy(L["plan"])
