"""Why the finite-temperature doubling expansion is kept on the mixed path.

Two alternative ways to evaluate the density at a given mu are measured here
with the oracle alone:

* Zero-temperature grand-canonical purification (McWeeny iteration towards
  the step function theta(mu - h)) is exact only where every subgraph has a
  gap around mu.  On a 1,000-water box partitioned like the benchmark
  workload (10-water grid cores, halos from one adaptive round at
  tau = 1e-3, non-orthogonal model, kT 0.1 eV), truncated halos put
  subgraph levels within kT of mu, and the collected zero-temperature count
  2 sum_k w_k theta(mu - lam_k) misses the electron count by more than
  1e-4 e at every mu between the nearest collected levels below and above
  mu, so no chemical potential reproduces the finite-temperature result.
* A Chebyshev expansion of the Fermi function over the spectral interval
  (for Paterson-Stockmeyer evaluation) needs a degree in the thousands for
  the accuracy of the doubling expansion at beta R = 270 (R = 27 eV, the
  half-width of the benchmark spectra about mu): about 2 sqrt(degree)
  products and sqrt(degree) stored powers combined per block, against 44
  products for six doublings.
"""
import numpy as np
import pytest
from numpy.polynomial import chebyshev as C

import waterbox
from oracle import graph as og
from oracle import model as om
from oracle import solve as osv


@pytest.mark.slow
def test_zero_temperature_count_misses_electron_count_in_the_gap():
    box = waterbox.water_box(1000, 3)
    L = box.box[0]
    m = om.TBModel(orthogonal=False, kT=0.1)
    rp, col = om.neighbour_list_kdtree(box.pos, L)
    core, nco = og.grid_cores(box.pos, box.anchor, L, (5, 5, 4))
    subs = og.extract_subgraphs(rp, col, core, nco)
    res = osv.solve_system(box.pos, box.species, L, m, subs)
    gd = og.condensed_dm(subs, res.d_core, box.species, box.n_atoms)
    g = og.graph_union(box.n_atoms, (rp, col), og.graph_dm(gd, 1e-3))
    subs = og.extract_subgraphs(g[0], g[1], core, nco)
    res = osv.solve_system(box.pos, box.species, L, m, subs)
    n_e = 8.0 * 1000
    lam = np.concatenate([s.lam for s in res.sols])
    w = np.concatenate([s.w for s in res.sols])
    below, above = lam[lam < res.mu].max(), lam[lam > res.mu].min()
    # a level within kT of mu: its finite-temperature occupation is fractional
    assert np.abs(lam - res.mu).min() < m.kT
    # the finite-temperature count meets n_e at the oracle's mu ...
    assert abs(osv.electron_count(res.sols, res.mu, m.beta) - n_e) < 1e-8
    # ... the zero-temperature count, constant between the two levels, does not
    for mu in np.linspace(below, above, 9)[1:-1]:
        n0 = 2.0 * w[lam < mu].sum()
        assert abs(n0 - n_e) > 1e-4


def test_chebyshev_degree_for_the_fermi_function():
    beta, R = 10.0, 27.0
    x = np.linspace(-1.0, 1.0, 100001)
    fermi = lambda t: 0.5 * (1.0 - np.tanh(0.5 * beta * R * t))
    err = {d: np.abs(C.chebval(x, C.chebinterpolate(fermi, d)) - fermi(x)).max() for d in (400, 800, 1200)}
    # the error falls only about tenfold per 100 degrees
    assert err[400] > 1e-3 and err[800] > 1e-5 and err[1200] > 1e-7
    assert err[1200] < err[800] < err[400]
