"""gdm_ewald_potential_noalloc (working memory in a fixed device array of the
library, no allocation) against gdm_ewald_potential on the same inputs: two
calls in a row, the second on a smaller system, plus the oracle's potential
and the host-side k_max limit."""
import numpy as np
import pytest
import torch

import waterbox
from oracle import ewald as oew
from paper_2606_03140_amd._lib import GDMError
from tests.gpu_common import ctx, log, system_of

pytestmark = pytest.mark.gpu

U_EV = (0.5 * 27.211386, 0.4 * 27.211386)


def _case(c, nw, seed, screened):
    from paper_2606_03140_amd import scc
    box = waterbox.water_box(nw, seed)
    sysm = system_of(box)
    q = np.random.default_rng(seed).normal(0.0, 1.0, size=len(box.species))
    q -= q.mean()
    qd = torch.as_tensor(q).to("cuda")
    ew = scc.ewald_setup(c, sysm)
    tau = scc.slater_tau(U_EV) if screened else None
    V_ref = c.ewald_potential(sysm, ew.graph, ew.rcut, ew.eta, ew.k_max, U_EV, qd, tau=tau)
    V = torch.full_like(V_ref, float("nan"))
    c.ewald_potential_noalloc(sysm, ew.graph, ew.rcut, ew.eta, ew.k_max, U_EV, qd, tau=tau, out=V)
    torch.cuda.synchronize()
    c.check()
    err = float((V - V_ref).abs().max())
    ref = oew.coulomb_potential(box.pos, box.species, q, box.box[0], np.array(U_EV), screened=screened,
                                short_cut=ew.rcut)
    err_o = float(np.abs(V.cpu().numpy() - ref).max())
    log(f"  {nw} waters k_max {ew.k_max} screened={screened}: max|V - allocating| {err:.1e} eV, "
        f"max|V - oracle| {err_o:.1e} eV")
    assert torch.isfinite(V).all()
    assert err < 1e-9
    assert err_o < 1e-8
    return sysm, ew, qd


def test_ewald_noalloc_matches_allocating_entry_point():
    c = ctx()
    log("Ewald potential without allocation vs the allocating entry point")
    _case(c, 300, 21, True)                  # larger first
    sysm, ew, qd = _case(c, 96, 1, False)    # then smaller: the scratch keeps the first call's contents
    with pytest.raises(GDMError) as e:
        c.ewald_potential_noalloc(sysm, ew.graph, ew.rcut, ew.eta, 33, U_EV, qd)
    assert e.value.code == -1
