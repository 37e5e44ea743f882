"""Test helpers: move packed image batches between numpy and device tensors.
No part of the method's arithmetic lives here."""
from __future__ import annotations

import numpy as np

from synth import pack_images


class Batch:
    def __init__(self, images: list[np.ndarray], align: int = 16):
        import torch
        self.images = images
        self.buf, self.h, self.w, self.p, self.o = pack_images(images, align_elems=align, pitch_multiple=align)
        self.dtype = self.buf.dtype
        self.dev = torch.from_numpy(self.buf.copy()).cuda()
        self.blocks = [((h + 15) // 16) * ((w + 15) // 16) for h, w in zip(self.h, self.w)]
        self.block_begin = np.concatenate([[0], np.cumsum(self.blocks)]).astype(np.int64)

    @property
    def n_blocks(self) -> int:
        return int(self.block_begin[-1])

    def plan(self, **kw):
        import paper_1606_05562_amd as A
        in_dtype = A.U8 if self.dtype == np.uint8 else A.I16
        return A.Plan(self.h, self.w, self.p, self.o, in_dtype=in_dtype, **kw)

    def empty_like_images(self, np_dtype, fill=0):
        import torch
        tdt = {np.uint8: torch.uint8, np.int16: torch.int16, np.float32: torch.float32}[np_dtype]
        return torch.full((len(self.buf),), fill, dtype=tdt, device="cuda")

    def unpack(self, dev_tensor) -> list[np.ndarray]:
        flat = dev_tensor.cpu().numpy()
        out = []
        for h, w, p, o in zip(self.h, self.w, self.p, self.o):
            out.append(flat[o:o + h * p].reshape(h, p)[:, :w].copy())
        return out

    def coef_tensor(self, torch_dtype):
        import torch
        return torch.zeros((self.n_blocks * 256,), dtype=torch_dtype, device="cuda")

    def split_coef(self, dev_tensor) -> list[np.ndarray]:
        flat = dev_tensor.cpu().numpy().reshape(-1, 16, 16)
        return [flat[self.block_begin[i]:self.block_begin[i + 1]] for i in range(len(self.images))]
