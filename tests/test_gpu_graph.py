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


def test_whole_fp64_solve_replays_from_a_hip_graph():
    """FP64 path with device outputs (gdm_set_mu_outputs): gather, Cholesky,
    eigensolver, mu search, density at the device mu and charges captured in
    one graph.  H is overwritten in place with the Hamiltonians of three SCC
    potentials; each replay must equal the eager solve of that H bit for bit
    (mu and N included), and the device mu must equal the host-output
    search's."""
    from paper_2606_03140_amd import pipeline
    from paper_2606_03140_amd._lib import Context
    prec = pipeline.FP64_EIG
    log("hipGraph capture of the whole FP64 solve (device mu), 96 waters, three potentials")
    hp = _hip()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        c = Context(0)
        box = waterbox.water_box(96, 1)
        sysm = system_of(box)
        tb = tb_params(False)
        part = pipeline.cutoff_partition(c, sysm, tb, (2, 2, 2))
        gen = torch.Generator().manual_seed(7)
        Hs = []
        for _ in range(3):
            V = (0.3 * torch.randn(sysm.n_atoms, generator=gen, dtype=torch.float64)).to(c.dev)
            Hs.append(c.build_hs(sysm, tb, part.nbr, V)[0])
        H, S = c.build_hs(sysm, tb, part.nbr)
        c.plan(part.sg, prec)
        c.set_mu_outputs(True)
        mu_t = torch.zeros(1, dtype=torch.float64, device=c.dev)
        n_t = torch.zeros_like(mu_t)
        D = torch.empty(int(part.sg.dcore_off[-1]), dtype=torch.float64, device=c.dev)
        q = torch.empty(sysm.n_atoms, dtype=torch.float64, device=c.dev)

        def solve():
            c.find_mu_device(sysm, part.sg, part.nbr, H, S, 0.1, prec, mu_t, n_t)
            c.subgraph_density_dmu(part.sg, mu_t, 0.1, prec, D)
            c.mulliken_charges(sysm, part.sg, part.nbr, S, D, out=q)

        refs = []
        for Hk in Hs:
            H.copy_(Hk)
            solve()
            c.check()
            refs.append((mu_t.clone(), n_t.clone(), D.clone(), q.clone()))
        torch.cuda.synchronize()
        # the device scalars hold the same search result as the host outputs
        c.set_mu_outputs(False)
        H.copy_(Hs[0])
        mu_h, n_h = c.find_mu(sysm, part.sg, part.nbr, H, S, 0.1, prec)
        assert mu_h == float(refs[0][0]) and n_h == float(refs[0][1])
        assert abs(n_h - sysm.n_electrons) < 1e-6 * sysm.n_electrons
        c.set_mu_outputs(True)
        torch.cuda.synchronize()
        st = C.c_void_p(side.cuda_stream)
        assert hp.hipStreamBeginCapture(st, _CAPTURE_RELAXED) == 0
        graph = C.c_void_p()
        try:
            solve()
        finally:
            rc_end = hp.hipStreamEndCapture(st, C.byref(graph))
        assert rc_end == 0
        exe = C.c_void_p()
        assert hp.hipGraphInstantiate(C.byref(exe), graph, None, None, 0) == 0
        try:
            for k, Hk in enumerate(Hs):
                H.copy_(Hk)
                for t in (mu_t, n_t, D, q):
                    t.fill_(float("nan"))
                assert hp.hipGraphLaunch(exe, st) == 0
                assert hp.hipStreamSynchronize(st) == 0
                c.check()
                mu_r, n_r, D_r, q_r = refs[k]
                log(f"  potential {k}: mu {float(mu_t):.9f} (eager {float(mu_r):.9f}), N {float(n_t):.9f}, "
                    f"max|q - eager| {float((q - q_r).abs().max()):.1e}")
                assert torch.equal(mu_t, mu_r) and torch.equal(n_t, n_r)
                assert torch.equal(D, D_r) and torch.equal(q, q_r)
            assert not torch.equal(refs[0][3], refs[1][3])
        finally:
            hp.hipGraphExecDestroy(exe)
            hp.hipGraphDestroy(graph)
            torch.cuda.synchronize()
            c.close()


def test_whole_mixed_solve_replays_from_a_hip_graph():
    """Mixed path with device outputs: the chemical-potential search runs a
    fixed number of passes and doublings whose launches are predicated on the
    device (gdm_set_mixed_capture), so gather, inverse overlap, expansion
    passes, mu, density at the device mu and charges capture into one graph.
    Each replay, with H overwritten by three SCC potentials, must equal the
    eager device-side solve bit for bit, and that solve must equal the
    host-driven search when it takes no more passes than were launched."""
    from paper_2606_03140_amd import pipeline
    from paper_2606_03140_amd._lib import Context, GDMError
    prec = pipeline.MIXED_F16
    log("hipGraph capture of the whole mixed solve (device mu), 96 waters, three potentials")
    hp = _hip()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        c = Context(0)
        box = waterbox.water_box(96, 1)
        sysm = system_of(box)
        tb = tb_params(False)
        part = pipeline.cutoff_partition(c, sysm, tb, (2, 2, 2))
        gen = torch.Generator().manual_seed(7)
        Hs = []
        for _ in range(3):
            V = (0.3 * torch.randn(sysm.n_atoms, generator=gen, dtype=torch.float64)).to(c.dev)
            Hs.append(c.build_hs(sysm, tb, part.nbr, V)[0])
        H, S = c.build_hs(sysm, tb, part.nbr)
        c.plan(part.sg, prec)
        # the charge response's recording is host-driven only
        c.set_response(8)
        c.set_mu_outputs(True)
        mu_t = torch.full((1,), float("nan"), dtype=torch.float64, device=c.dev)
        n_t = torch.zeros_like(mu_t)
        with pytest.raises(GDMError) as e:
            c.find_mu_device(sysm, part.sg, part.nbr, H, S, 0.1, prec, mu_t, n_t, mu_guess=-7.0, tol_N=1e-6)
        assert e.value.code == -1
        c.set_response(0)
        c.plan(part.sg, prec)
        c.set_mixed_capture(6, 10)
        D = torch.empty(int(part.sg.dcore_off[-1]), dtype=torch.float64, device=c.dev)
        q = torch.empty(sysm.n_atoms, dtype=torch.float64, device=c.dev)

        def solve():
            mu_t.fill_(float("nan"))          # start every solve from the host guess
            c.find_mu_device(sysm, part.sg, part.nbr, H, S, 0.1, prec, mu_t, n_t, mu_guess=-7.0, tol_N=1e-6)
            c.subgraph_density_dmu(part.sg, mu_t, 0.1, prec, D)
            c.mulliken_charges(sysm, part.sg, part.nbr, S, D, out=q)

        refs = []
        for Hk in Hs:
            H.copy_(Hk)
            solve()
            c.check()
            st = c.mixed_stats()
            refs.append((mu_t.clone(), n_t.clone(), D.clone(), q.clone(), st["passes"], st["n_doublings"]))
            log(f"  eager device search: mu {float(mu_t):.9f} N {float(n_t):.9f} passes {st['passes']} "
                f"n_d {st['n_doublings']}")
            assert abs(float(n_t) - sysm.n_electrons) <= 1e-7 * sysm.n_electrons
        torch.cuda.synchronize()
        # the host-driven search does the same arithmetic
        c.set_mu_outputs(False)
        H.copy_(Hs[0])
        mu_h, n_h = c.find_mu(sysm, part.sg, part.nbr, H, S, 0.1, prec, -7.0, 1e-6)
        sth = c.mixed_stats()
        log(f"  host search: mu {mu_h:.9f} passes {sth['passes']}")
        if sth["passes"] <= 6:
            assert mu_h == float(refs[0][0]) and n_h == float(refs[0][1])
        c.set_mu_outputs(True)
        torch.cuda.synchronize()
        stc = C.c_void_p(side.cuda_stream)
        assert hp.hipStreamBeginCapture(stc, _CAPTURE_RELAXED) == 0
        graph = C.c_void_p()
        try:
            solve()
        finally:
            rc_end = hp.hipStreamEndCapture(stc, C.byref(graph))
        assert rc_end == 0
        exe = C.c_void_p()
        assert hp.hipGraphInstantiate(C.byref(exe), graph, None, None, 0) == 0
        try:
            for k, Hk in enumerate(Hs):
                H.copy_(Hk)
                for t in (n_t, D, q):
                    t.fill_(float("nan"))
                assert hp.hipGraphLaunch(exe, stc) == 0
                assert hp.hipStreamSynchronize(stc) == 0
                c.check()
                mu_r, n_r, D_r, q_r, _, _ = refs[k]
                log(f"  potential {k}: mu {float(mu_t):.9f} (eager {float(mu_r):.9f}), N {float(n_t):.9f}, "
                    f"max|q - eager| {float((q - q_r).abs().max()):.1e}")
                assert torch.equal(mu_t, mu_r) and torch.equal(n_t, n_r)
                assert torch.equal(D, D_r) and torch.equal(q, q_r)
                # eager host-driven work between the replays
                c.set_mu_outputs(False)
                c.find_mu(sysm, part.sg, part.nbr, H, S, 0.1, prec, -7.0, 1e-6)
                c.set_mu_outputs(True)
                torch.cuda.synchronize()
            assert not torch.equal(refs[0][3], refs[1][3])
        finally:
            hp.hipGraphExecDestroy(exe)
            hp.hipGraphDestroy(graph)
            torch.cuda.synchronize()
            c.set_mu_outputs(False)
            c.close()
