"""Renderer adapter over the HIP library (GPU tests): device buffers come
from torch, every computation runs in libamr.so."""
import numpy as np
import torch

import paper_1210_8014_amd as amr


def stream():
    return torch.cuda.current_stream().cuda_stream


class GpuRenderer:
    def __init__(self, leaves, restrict=None, variant=-1):
        self.T = amr.Tree(leaves, restrict=restrict)
        self.variant = variant

    def camera(self, d):
        return amr.set_camera(d, self.T)

    def full(self, cam, op, field=0, weight=0, los=False, variant=None):
        n = cam.W * cam.H
        out = torch.empty(n, dtype=torch.float32, device="cuda")
        aux = torch.empty(n, dtype=torch.float32, device="cuda") if op == amr.WMEAN else None
        amr.render(self.T, cam, op, out, aux, field=field, weight=weight, los=los,
                   variant=self.variant if variant is None else variant)
        torch.cuda.synchronize()
        return out.cpu().numpy(), (aux.cpu().numpy() if aux is not None else None)

    def counts(self, cam):
        n = cam.W * cam.H
        cnt = torch.empty(n, dtype=torch.int32, device="cuda")
        tot = torch.empty(1, dtype=torch.int64, device="cuda")
        amr.count_segments(self.T, cam, tot, cnt)
        torch.cuda.synchronize()
        return cnt.cpu().numpy(), int(tot.item())

    def render(self, cam, op, field=0, weight=0, los=False, rays=None):
        out, aux = self.full(cam, op, field, weight, los)
        cnt, _ = self.counts(cam)
        if rays is not None:
            out, cnt = out[rays], cnt[rays]
            aux = aux[rays] if aux is not None else None
        return out, aux, cnt

    def trace(self, cam, rays):
        r = torch.as_tensor(np.ascontiguousarray(rays, np.int64), device="cuda")
        cnt = torch.empty(r.numel(), dtype=torch.int32, device="cuda")
        amr.count_rays(self.T, cam, r, cnt)
        torch.cuda.synchronize()
        c = cnt.cpu().numpy().astype(np.int64)
        offs = np.zeros(len(rays) + 1, np.int64)
        offs[1:] = np.cumsum(c)
        cells = torch.zeros((max(int(offs[-1]), 1), 4), dtype=torch.int32, device="cuda")
        amr.trace_rays(self.T, cam, r, torch.as_tensor(offs, device="cuda"), cells)
        torch.cuda.synchronize()
        return offs, cells.cpu().numpy()[:int(offs[-1])]
