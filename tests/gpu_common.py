"""Shared helpers of the GPU parity tests (imported by tests only)."""
import numpy as np
import torch

import waterbox
from oracle import model as omodel
from paper_2606_03140_amd import _lib
from paper_2606_03140_amd._lib import Context, System, TBParams

_CTX = None


def ctx():
    global _CTX
    if _CTX is None:
        _CTX = Context(0)
    return _CTX


def system_of(box: waterbox.WaterBox) -> System:
    return System(box.pos, box.species, box.anchor, box.box)


def oracle_model(orthogonal: bool, kT: float = 0.1) -> omodel.TBModel:
    return omodel.TBModel(orthogonal=orthogonal, kT=kT)


def tb_params(orthogonal: bool) -> TBParams:
    return TBParams(orthogonal=orthogonal)


def csr_host(g):
    return g.row_ptr.cpu().numpy().astype(np.int64), g.col.cpu().numpy().astype(np.int64)


def unpack_dcore(sg, D):
    D = D.cpu().numpy()
    out = []
    for s in range(sg.n_sub):
        n, nc = int(sg.norb[s]), int(sg.ncore_orb[s])
        out.append(D[sg.dcore_off[s]:sg.dcore_off[s + 1]].reshape(nc, n))
    return out


def pack_dcore(dcs):
    return torch.as_tensor(np.concatenate([d.ravel() for d in dcs])).to("cuda")


def log(msg):
    print(msg, flush=True)
