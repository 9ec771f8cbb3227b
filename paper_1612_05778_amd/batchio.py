"""Packing many products into single device buffers for batched calls.

All operands go into one int64 device tensor and all outputs into another; each
product's zpm_job points at its slices.  This keeps the number of allocations and
host-to-device copies independent of the number of products.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _native as nat
from .api import out_words


class PackedBatch:
    def __init__(self, prods, device="cuda"):
        self.prods = prods
        n = len(prods)
        in_words = sum(p.a.size + p.b.size for p in prods)
        self.wcs = [out_words(p.da, p.Na, p.db, p.Nb) for p in prods]
        self.nouts = [p.da + p.db - 1 for p in prods]
        out_words_total = sum(w * m for w, m in zip(self.wcs, self.nouts))
        host = np.empty(in_words, dtype=np.uint64)
        self.a_off, self.b_off, self.c_off = [], [], []
        pos = 0
        for p in prods:
            self.a_off.append(pos)
            host[pos:pos + p.a.size] = p.a.ravel()
            pos += p.a.size
            self.b_off.append(pos)
            host[pos:pos + p.b.size] = p.b.ravel()
            pos += p.b.size
        pos = 0
        for w, m in zip(self.wcs, self.nouts):
            self.c_off.append(pos)
            pos += w * m
        self.inputs = torch.from_numpy(host.view(np.int64)).to(device)
        self.outputs = torch.zeros(max(out_words_total, 1), dtype=torch.int64, device=device)
        ia, io = self.inputs.data_ptr(), self.outputs.data_ptr()
        self.jobs = (nat.Job * max(n, 1))()
        for i, p in enumerate(prods):
            j = self.jobs[i]
            j.a, j.da, j.Na = ia + 8 * self.a_off[i], p.da, p.Na
            j.b, j.db, j.Nb = ia + 8 * self.b_off[i], p.db, p.Nb
            j.c, j.wc = io + 8 * self.c_off[i], self.wcs[i]
        self.n = n

    def out(self, i: int) -> torch.Tensor:
        o = self.c_off[i]
        return self.outputs[o:o + self.wcs[i] * self.nouts[i]].view(self.nouts[i], self.wcs[i])

    def bits(self) -> int:
        from .workmodel import product_bits
        return sum(product_bits(p.da, p.Na, p.db, p.Nb) for p in self.prods)
