"""hipGraph capture of the calls that follow the chemical potential.

After gdm_find_mu, gdm_subgraph_density and gdm_mulliken_charges enqueue
kernels only: no allocation, no host synchronisation, no memset.  Here they
are captured on the context's stream (a non-default torch stream), the graph
is instantiated and replayed three times, with eager library work (a density
at another mu, into another buffer) and synchronisations between the replays,
and every replay must reproduce the eager D core rows and charges bit for bit
(the same kernels with the same arguments; each output element has a single
writer, so there is no order dependence).  A replay reads the context's state
from the last gdm_find_mu, which the eager work in between does not change.
Both precisions, 96 waters, non-orthogonal model, 2x2x2 cores.
"""
import ctypes as C

import pytest
import torch

import waterbox
from tests.gpu_common import log, system_of, tb_params

pytestmark = pytest.mark.gpu

_CAPTURE_RELAXED = 2          # hipStreamCaptureModeRelaxed


def _hip():
    # the HIP runtime torch has already loaded (libgdm resolves to the same one)
    h = C.CDLL("libamdhip64.so.7")
    h.hipStreamBeginCapture.argtypes = [C.c_void_p, C.c_int]
    h.hipStreamEndCapture.argtypes = [C.c_void_p, C.POINTER(C.c_void_p)]
    h.hipGraphInstantiate.argtypes = [C.POINTER(C.c_void_p), C.c_void_p, C.c_void_p, C.c_char_p, C.c_size_t]
    h.hipGraphLaunch.argtypes = [C.c_void_p, C.c_void_p]
    h.hipGraphExecDestroy.argtypes = [C.c_void_p]
    h.hipGraphDestroy.argtypes = [C.c_void_p]
    h.hipStreamSynchronize.argtypes = [C.c_void_p]
    return h


@pytest.mark.parametrize("path", ["fp64", "mixed"])
def test_density_and_charges_replay_from_a_hip_graph(path):
    from paper_2606_03140_amd import pipeline
    from paper_2606_03140_amd._lib import Context
    prec = {"fp64": pipeline.FP64_EIG, "mixed": pipeline.MIXED_F16}[path]
    log(f"hipGraph capture of density + Mulliken, {path} path, 96 waters")
    hp = _hip()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        c = Context(0)                       # bound to the side stream
        box = waterbox.water_box(96, 1)
        sysm = system_of(box)
        tb = tb_params(False)
        part = pipeline.cutoff_partition(c, sysm, tb, (2, 2, 2))
        H, S = c.build_hs(sysm, tb, part.nbr)
        c.plan(part.sg, prec)
        mu, n = c.find_mu(sysm, part.sg, part.nbr, H, S, 0.1, prec, -7.0, 1e-6)
        D_ref = c.subgraph_density(part.sg, mu, 0.1, prec)
        q_ref = c.mulliken_charges(sysm, part.sg, part.nbr, S, D_ref)
        D = torch.full_like(D_ref, float("nan"))
        q = torch.full_like(q_ref, float("nan"))
        D_other = torch.empty_like(D_ref)
        torch.cuda.synchronize()
        st = C.c_void_p(side.cuda_stream)
        assert hp.hipStreamBeginCapture(st, _CAPTURE_RELAXED) == 0
        graph = C.c_void_p()
        try:
            c.subgraph_density(part.sg, mu, 0.1, prec, out=D)
            c.mulliken_charges(sysm, part.sg, part.nbr, S, D, out=q)
        finally:
            rc_end = hp.hipStreamEndCapture(st, C.byref(graph))
        assert rc_end == 0
        exe = C.c_void_p()
        assert hp.hipGraphInstantiate(C.byref(exe), graph, None, None, 0) == 0
        try:
            # capture enqueued nothing: the outputs are still NaN
            torch.cuda.synchronize()
            assert torch.isnan(D).all() and torch.isnan(q).all()
            for k in range(3):
                D.fill_(float("nan"))
                q.fill_(float("nan"))
                assert hp.hipGraphLaunch(exe, st) == 0
                assert hp.hipStreamSynchronize(st) == 0
                c.check()
                log(f"  replay {k}: max|D - eager| {float((D - D_ref).abs().max()):.1e}, "
                    f"max|q - eager| {float((q - q_ref).abs().max()):.1e}")
                assert torch.equal(D, D_ref) and torch.equal(q, q_ref)
                # eager work between replays
                c.subgraph_density(part.sg, mu + 0.05, 0.1, prec, out=D_other)
                torch.cuda.synchronize()
                assert not torch.equal(D_other, D_ref)
        finally:
            hp.hipGraphExecDestroy(exe)
            hp.hipGraphDestroy(graph)
            torch.cuda.synchronize()
            c.close()
    log(f"  mu {mu:.6f}, N {n:.9f}, {part.sg.n_sub} subgraphs")
